// VDI generation on the GPU (paper Section 3: supersegments by Eq. 1 along
// each generating ray of V_O; supplement Alg. S1: per-ray bisection of the
// sensitivity gamma so that a ray yields at most N_S supersegments).
//
// One thread per generating ray, FP64 throughout, every expression in the
// order written and without contraction into fused multiply-adds, so that the
// comparisons deciding supersegment boundaries come out as the same arithmetic
// does on a CPU.  A thread cannot keep a ray's samples, so each pass over the
// ray (direct volume rendering to find where early termination ends it, each
// counting pass of the bisection, the final capped split) samples the volume
// again: trilinear interpolation of cell-centred voxels, transfer function,
// opacity corrected to the sample length.
#include <hip/hip_runtime.h>

#include <math.h>
#include <string.h>

#include <algorithm>

#include "vdi_internal.h"

namespace vdi {
namespace {

constexpr double kGenTTerm = 1e-5;  // early ray termination of the generating rays

struct GenCam {
    double eye[3], F[3], R[3], U[3], tanh_, aspect, near_;
    int W, H;
};

struct GenVol {
    int nx, ny, nz, is_u16;
    const void *data;
    double bmin[3], bmax[3];
    __host__ __device__ int n(int a) const { return a == 0 ? nx : (a == 1 ? ny : nz); }
};

struct GenParams {
    GenCam cam;
    GenVol vol;
    int NS, tf, maxs, delta;
    double ds, gamma;  // gamma > 0: fixed
};

// FP64 pow, out of line on the device: both call sites (a sample's opacity
// and the criterion's rescaled opacity) then share one copy and its
// registers, and the kernel spills less (4-8% faster than inlined).
#ifdef __HIP_DEVICE_COMPILE__
__device__ __noinline__ double gen_pow(double x, double y) { return pow(x, y); }
#else
__host__ inline double gen_pow(double x, double y) { return pow(x, y); }
#endif

struct Sample {
    double c[3], a;  // straight colour, opacity corrected to the sample length
    double v;        // interpolated scalar
};

// A lane's cache of its ray's first K samples, (v, a) of sample q at
// p[q * stride]: the passes after the first read them back instead of
// sampling the volume again.  K = 0: no cache.
struct SampleCache {
    double2 *p;
    int K, stride;
};

struct Seg {
    double ts, te, C[3], A;  // t-range, premultiplied colour, opacity
};

__host__ __device__ inline double clamp01(double v)
{
#pragma clang fp contract(off)
    return v < 0.0 ? 0.0 : (v > 1.0 ? 1.0 : v);
}

__host__ __device__ inline double voxel(const GenVol &v, int i, int j, int k)
{
#pragma clang fp contract(off)
    const size_t o = ((size_t)k * v.ny + j) * v.nx + i;
    return v.is_u16 ? (double)static_cast<const uint16_t *>(v.data)[o] * (1.0 / 65535.0)
                    : (double)static_cast<const float *>(v.data)[o];
}

__host__ __device__ inline int clampi(int x, int lo, int hi) { return x < lo ? lo : (x > hi ? hi : x); }

// Trilinear interpolation of cell-centred voxels, clamped to the edge.
__host__ __device__ inline double sample_tri(const GenVol &v, const double *P)
{
#pragma clang fp contract(off)
    const int n[3] = {v.nx, v.ny, v.nz};
    double w[3];
    int i0[3], i1[3];
    for (int a = 0; a < 3; ++a) {
        const double u = (P[a] - v.bmin[a]) / (v.bmax[a] - v.bmin[a]) * n[a] - 0.5;
        const double f = floor(u);
        w[a] = u - f;
        i0[a] = clampi((int)f, 0, n[a] - 1);
        i1[a] = clampi((int)f + 1, 0, n[a] - 1);
    }
    const double c00 = voxel(v, i0[0], i0[1], i0[2]) * (1 - w[0]) + voxel(v, i1[0], i0[1], i0[2]) * w[0];
    const double c10 = voxel(v, i0[0], i1[1], i0[2]) * (1 - w[0]) + voxel(v, i1[0], i1[1], i0[2]) * w[0];
    const double c01 = voxel(v, i0[0], i0[1], i1[2]) * (1 - w[0]) + voxel(v, i1[0], i0[1], i1[2]) * w[0];
    const double c11 = voxel(v, i0[0], i1[1], i1[2]) * (1 - w[0]) + voxel(v, i1[0], i1[1], i1[2]) * w[0];
    const double c0 = c00 * (1 - w[1]) + c10 * w[1], c1 = c01 * (1 - w[1]) + c11 * w[1];
    return c0 * (1 - w[2]) + c1 * w[2];
}

// The two transfer functions of the synthetic workloads (VDI_TF_*).
__host__ __device__ inline void tf_eval(int tf, double v, double *c, double &a)
{
#pragma clang fp contract(off)
    if (tf == VDI_TF_RAMP) {
        c[0] = v;
        c[1] = 0.25 + 0.5 * v;
        c[2] = 1.0 - v;
        a = 0.2 * clamp01((v - 0.05) / 0.95);
        return;
    }
    const double kv[4] = {0.0, 0.25, 0.55, 1.0};
    const double ka[4] = {0.0, 0.0, 0.04, 0.12};
    const double kc[4][3] = {{0.1, 0.2, 0.8}, {0.1, 0.7, 0.9}, {0.95, 0.9, 0.3}, {0.9, 0.15, 0.1}};
    v = clamp01(v);
    const int s = v < kv[1] ? 0 : (v < kv[2] ? 1 : 2);
    const double u = (v - kv[s]) / (kv[s + 1] - kv[s]);
    for (int m = 0; m < 3; ++m) c[m] = kc[s][m] + u * (kc[s + 1][m] - kc[s][m]);
    a = ka[s] + u * (ka[s + 1] - ka[s]);
}

// Sample q of a ray (midpoint of [t0 + q len, t0 + (q + 1) len]).
__host__ __device__ inline Sample take_sample(const GenParams &G, const double *d, double t0, double len, int q)
{
#pragma clang fp contract(off)
    const double tm = t0 + (q + 0.5) * len;
    double P[3];
    for (int a = 0; a < 3; ++a) P[a] = G.cam.eye[a] + tm * d[a];
    const double v = sample_tri(G.vol, P);
    Sample s;
    double atf;
    tf_eval(G.tf, v, s.c, atf);
    s.a = atf > 0.0 ? 1.0 - gen_pow(1.0 - atf, len / G.ds) : 0.0;
    s.v = v;
    return s;
}

// Sample q from the cache when it holds it (the same doubles: the colour is
// the transfer function of the same v), else from the volume.
__host__ __device__ inline Sample cached_sample(const GenParams &G, const SampleCache &C, const double *d, double t0,
                                                double len, int q)
{
    if (q < C.K) {
        const double2 e = C.p[(size_t)q * C.stride];
        Sample s;
        double atf;
        tf_eval(G.tf, e.x, s.c, atf);
        s.a = e.y;
        s.v = e.x;
        return s;
    }
    return take_sample(G, d, t0, len, q);
}

// Split the first ns samples of a ray into supersegments with sensitivity
// gamma (Eq. 1).  cap == 0: count only.  cap > 0: at most cap supersegments;
// once cap - 1 are closed the last one takes every remaining non-transparent
// sample, across gaps.  Eq. 1 compares the open supersegment's straight colour
// times its opacity normalised to one sample length with the next sample's
// colour times its opacity.  With WRITE, supersegment j goes to slot j of
// list li (depths as V_O view depth f = t cos(theta), b likewise).
template <bool WRITE>
__host__ __device__ inline int split_ray(const GenParams &G, const SampleCache &C, const double *d, double cth, double t0,
                                         double len, int ns, double gamma, int cap, size_t li, size_t plane,
                                         float2 *depth, float4 *rgba)
{
#pragma clang fp contract(off)
    int nclosed = 0;
    bool open = false;
    Seg cur = {0.0, 0.0, {0.0, 0.0, 0.0}, 0.0};
    auto close = [&]() {
        if constexpr (WRITE) {
            float f = (float)(cur.ts * cth), b = (float)(cur.te * cth);
            if (!(b > f)) b = nextafterf(f, INFINITY);
            const size_t o = (size_t)nclosed * plane + li;
            depth[o] = make_float2(f, b);
            const double A = cur.A;
            rgba[o] = make_float4((float)(cur.C[0] / A), (float)(cur.C[1] / A), (float)(cur.C[2] / A), (float)A);
        }
        ++nclosed;
        open = false;
    };
    for (int q = 0; q < ns; ++q) {
        const Sample s = cached_sample(G, C, d, t0, len, q);
        const bool last = cap > 0 && nclosed == cap - 1;
        if (s.a == 0.0) {
            if (open && !last) close();
            continue;
        }
        const double qs = t0 + q * len, qe = t0 + (q + 1) * len;
        if (open && !last) {
            const double lenS = cur.te - cur.ts;
            const double abar = 1.0 - gen_pow(1.0 - cur.A, len / lenS);
            double d2 = 0.0;
            for (int m = 0; m < 3; ++m) {
                const double e = cur.C[m] / cur.A * abar - s.c[m] * s.a;
                d2 += e * e;
            }
            if (sqrt(d2) >= gamma) close();
        }
        if (!open) {
            cur.ts = qs;
            cur.te = qe;
            cur.A = s.a;
            for (int m = 0; m < 3; ++m) cur.C[m] = s.a * s.c[m];
            open = true;
            continue;
        }
        for (int m = 0; m < 3; ++m) cur.C[m] += (1.0 - cur.A) * s.a * s.c[m];
        cur.A += (1.0 - cur.A) * s.a;
        cur.te = qe;
    }
    if (open) close();
    return nclosed;
}

// Ray through the centre of pixel (px, py) of the camera, clipped to the
// AABB and the camera's near plane: unit direction d, cos(theta) = F.d and
// the parameter range [t0, t1] along d (false when empty).
__host__ __device__ inline bool ray_clip(const GenParams &G, int px, int py, double *d, double &cth, double &t0,
                                         double &t1)
{
#pragma clang fp contract(off)
    const int W = G.cam.W, H = G.cam.H;
    const double xc = -1.0 + (2.0 * px + 1.0) / W, yc = -1.0 + (2.0 * py + 1.0) / H;
    for (int a = 0; a < 3; ++a)
        d[a] = G.cam.F[a] + xc * G.cam.tanh_ * G.cam.aspect * G.cam.R[a] + yc * G.cam.tanh_ * G.cam.U[a];
    const double nrm = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
    for (int a = 0; a < 3; ++a) d[a] /= nrm;
    cth = G.cam.F[0] * d[0] + G.cam.F[1] * d[1] + G.cam.F[2] * d[2];
    double lo = G.cam.near_ / cth, hi = INFINITY;
    for (int a = 0; a < 3; ++a) {
        if (fabs(d[a]) < 1e-300) {
            if (G.cam.eye[a] < G.vol.bmin[a] || G.cam.eye[a] > G.vol.bmax[a]) return false;
            continue;
        }
        double ta = (G.vol.bmin[a] - G.cam.eye[a]) / d[a], tb = (G.vol.bmax[a] - G.cam.eye[a]) / d[a];
        if (ta > tb) {
            const double t = ta;
            ta = tb;
            tb = t;
        }
        if (ta > lo) lo = ta;
        if (tb < hi) hi = tb;
    }
    t0 = lo;
    t1 = hi;
    return hi > lo;
}

// Number of equal samples over [t0, t1]: about one per ds, at least 1.
__host__ __device__ inline int sample_count(const GenParams &G, double t0, double t1)
{
#pragma clang fp contract(off)
    int N = (int)ceil((t1 - t0) / G.ds - 1e-9);
    if (N < 1) N = 1;
    if (N > G.maxs) N = G.maxs;
    return N;
}

// Sensitivity of one ray (supplement Alg. S1; bracket updates as read in
// the design notes).  count(g), the ray's supersegments at sensitivity g,
// does not grow with g; the search wants N_S - delta <= count(g) <= N_S.
// A first trial at 1e-5 stands if it gives at most N_S.  Otherwise the
// bracket (lo, hi) always has count(lo) > N_S, and hi is sqrt 3 or gives
// fewer than N_S - delta; each further trial halves it.  A bracket narrower
// than 1e-6 ends the search at hi, or at lo if the trial in hand gives no
// supersegment; so does the 25th trial.
template <typename Count>
__host__ __device__ double search_gamma(int NS, int delta, Count count)
{
#pragma clang fp contract(off)
    double lo = 1e-5;
    if (count(lo) <= NS) return lo;
    double hi = sqrt(3.0);
    int trials = 1;
    for (;;) {
        const double g = 0.5 * (lo + hi);
        const int c = count(g);
        ++trials;
        if (hi - lo < 1e-6) return c == 0 ? lo : hi;
        if (c > NS)
            lo = g;
        else if (c < NS - delta)
            hi = g;
        else
            return g;
        if (trials == 25) return hi;
    }
}

// The whole generation of list (px, py): ray, samples, gamma, supersegments.
__host__ __device__ inline void gen_ray(const GenParams &G, const SampleCache &C, int px, int py, uint8_t *count,
                                        float2 *depth, float4 *rgba, double *gamma_out)
{
#pragma clang fp contract(off)
    const int W = G.cam.W, H = G.cam.H;
    const size_t li = (size_t)py * W + px, plane = (size_t)W * H;
    double d[3], cth, t0, t1;
    const bool hit = ray_clip(G, px, py, d, cth, t0, t1);
    int n = 0;
    double gamma = 0.0;
    if (hit) {
        const int N = sample_count(G, t0, t1);
        const double len = (t1 - t0) / N;
        // Direct volume rendering front to back: where early termination ends the ray.
        double T = 1.0;
        int ns = 0;
        for (int q = 0; q < N; ++q) {
            const Sample s = take_sample(G, d, t0, len, q);
            if (q < C.K) C.p[(size_t)q * C.stride] = make_double2(s.v, s.a);
            ++ns;
            T *= 1.0 - s.a;
            if (T <= kGenTTerm) break;
        }
        if (G.gamma > 0.0) {
            gamma = G.gamma;
        } else {
            gamma = search_gamma(G.NS, G.delta, [&](double g) {
                return split_ray<false>(G, C, d, cth, t0, len, ns, g, 0, li, plane, nullptr, nullptr);
            });
        }
        n = split_ray<true>(G, C, d, cth, t0, len, ns, gamma, G.NS, li, plane, depth, rgba);
    }
    count[li] = (uint8_t)n;
    if (gamma_out) gamma_out[li] = gamma;
    for (int j = n; j < G.NS; ++j) {
        depth[(size_t)j * plane + li] = make_float2(0.0f, 0.0f);
        rgba[(size_t)j * plane + li] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    }
}

// Persistent wavefronts: each takes the next tile of 64 rays from `counter`
// (zero at launch) until none is left, and keeps the samples of its rays in
// its own cache region: [K][64 lanes] of (v, a), so that the 64 lanes, which
// step through a pass in lockstep, touch 1 KiB of consecutive memory per
// sample.  Samples beyond K are taken from the volume again.
constexpr size_t kGenCacheBytes = (size_t)4 << 30;  // at most this much cache in all
// A wavefront generates a tile of kGenTileW x kGenTileH rays: neighbouring
// rays in both directions see similar data, so their work differs less.
#ifndef VDI_GEN_TILE_W
#define VDI_GEN_TILE_W 8
#endif
constexpr int kGenTileW = VDI_GEN_TILE_W, kGenTileH = 64 / VDI_GEN_TILE_W;
#ifndef VDI_GEN_WAVES
#define VDI_GEN_WAVES 3  // wavefronts per SIMD the kernel is compiled for
#endif

__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(VDI_GEN_WAVES))) void k_generate(GenParams G, unsigned *__restrict__ counter, int ntiles,
                                                 double2 *__restrict__ cache, int K, uint8_t *__restrict__ count,
                                                 float2 *__restrict__ depth, float4 *__restrict__ rgba,
                                                 double *__restrict__ gamma_out)
{
    const int tiles_x = (G.cam.W + kGenTileW - 1) / kGenTileW;
    const SampleCache C = {cache + (size_t)blockIdx.x * K * 64 + threadIdx.x, K, 64};
    for (;;) {
        int tile = 0;
        if (threadIdx.x == 0) tile = (int)atomicAdd(counter, 1u);
        tile = __shfl(tile, 0);
        if (tile >= ntiles) break;
        const int px = (tile % tiles_x) * kGenTileW + (int)threadIdx.x % kGenTileW;
        const int py = (tile / tiles_x) * kGenTileH + (int)threadIdx.x / kGenTileW;
        if (px < G.cam.W && py < G.cam.H) gen_ray(G, C, px, py, count, depth, rgba, gamma_out);
    }
}

// ---------------------------------------------------------------------------
// Direct volume rendering (the image a VDI approximates; Section 6 compares
// VDI renderings against it): one lane per pixel of the camera, the samples
// and transfer function of generation, front-to-back emission-absorption with
// early termination at transmittance <= 1e-5.
// ---------------------------------------------------------------------------

// FP32 shading: the voxel coordinates u (FP64, cell-centred: voxel i at
// u = i) give the trilinear cell and weights; interpolation, transfer
// function, opacity and compositing run in FP32.
__device__ inline float sample_tri_f32(const GenVol &v, const double *u)
{
    const int n[3] = {v.nx, v.ny, v.nz};
    float w[3];
    int i0[3], i1[3];
    for (int a = 0; a < 3; ++a) {
        const double f = floor(u[a]);
        w[a] = (float)(u[a] - f);
        i0[a] = clampi((int)f, 0, n[a] - 1);
        i1[a] = clampi((int)f + 1, 0, n[a] - 1);
    }
    auto vx = [&](int i, int j, int k) { return (float)voxel(v, i, j, k); };
    const float c00 = vx(i0[0], i0[1], i0[2]) * (1 - w[0]) + vx(i1[0], i0[1], i0[2]) * w[0];
    const float c10 = vx(i0[0], i1[1], i0[2]) * (1 - w[0]) + vx(i1[0], i1[1], i0[2]) * w[0];
    const float c01 = vx(i0[0], i0[1], i1[2]) * (1 - w[0]) + vx(i1[0], i0[1], i1[2]) * w[0];
    const float c11 = vx(i0[0], i1[1], i1[2]) * (1 - w[0]) + vx(i1[0], i1[1], i1[2]) * w[0];
    const float c0 = c00 * (1 - w[1]) + c10 * w[1], c1 = c01 * (1 - w[1]) + c11 * w[1];
    return c0 * (1 - w[2]) + c1 * w[2];
}

__device__ inline void tf_eval_f32(int tf, float v, float *c, float &a)
{
    if (tf == VDI_TF_RAMP) {
        c[0] = v;
        c[1] = 0.25f + 0.5f * v;
        c[2] = 1.0f - v;
        a = 0.2f * fminf(fmaxf((v - 0.05f) / 0.95f, 0.0f), 1.0f);
        return;
    }
    const float kv[4] = {0.0f, 0.25f, 0.55f, 1.0f};
    const float ka[4] = {0.0f, 0.0f, 0.04f, 0.12f};
    const float kc[4][3] = {{0.1f, 0.2f, 0.8f}, {0.1f, 0.7f, 0.9f}, {0.95f, 0.9f, 0.3f}, {0.9f, 0.15f, 0.1f}};
    v = fminf(fmaxf(v, 0.0f), 1.0f);
    const int s = v < kv[1] ? 0 : (v < kv[2] ? 1 : 2);
    const float u = (v - kv[s]) / (kv[s + 1] - kv[s]);
    for (int m = 0; m < 3; ++m) c[m] = kc[s][m] + u * (kc[s + 1][m] - kc[s][m]);
    a = ka[s] + u * (ka[s + 1] - ka[s]);
}

template <bool F64>
__global__ __launch_bounds__(64) void k_dvr(GenParams G, float4 *__restrict__ out)
{
#pragma clang fp contract(off)
    const int px = blockIdx.x * 64 + threadIdx.x, py = blockIdx.y;
    if (px >= G.cam.W || py >= G.cam.H) return;
    double d[3], cth, t0, t1;
    float4 o = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    if (ray_clip(G, px, py, d, cth, t0, t1)) {
        const int N = sample_count(G, t0, t1);
        const double len = (t1 - t0) / N;
        if constexpr (F64) {
            double T = 1.0, acc[3] = {0.0, 0.0, 0.0};
            for (int q = 0; q < N; ++q) {
                const Sample s = take_sample(G, d, t0, len, q);
                for (int m = 0; m < 3; ++m) acc[m] += T * s.a * s.c[m];
                T *= 1.0 - s.a;
                if (T <= kGenTTerm) break;
            }
            o = make_float4((float)acc[0], (float)acc[1], (float)acc[2], (float)(1.0 - T));
        } else {
            // Opacity 1 - (1 - a)^r as 1 - 2^(r log2(1 - a)) with the hardware
            // base-2 exponential and logarithm.
            const float r = (float)(len / G.ds);
            // Voxel coordinate of sample q along each axis: u0 + q du (FP64).
            double u0[3], du[3];
            for (int a = 0; a < 3; ++a) {
                const double sc = G.vol.n(a) / (G.vol.bmax[a] - G.vol.bmin[a]);
                u0[a] = (G.cam.eye[a] + (t0 + 0.5 * len) * d[a] - G.vol.bmin[a]) * sc - 0.5;
                du[a] = len * d[a] * sc;
            }
            float T = 1.0f, acc[3] = {0.0f, 0.0f, 0.0f};
            for (int q = 0; q < N; ++q) {
                double u[3];
                for (int a = 0; a < 3; ++a) u[a] = u0[a] + q * du[a];
                float c[3], atf;
                tf_eval_f32(G.tf, sample_tri_f32(G.vol, u), c, atf);
                const float ap = atf > 0.0f ? 1.0f - __builtin_amdgcn_exp2f(r * __builtin_amdgcn_logf(1.0f - atf)) : 0.0f;
                for (int m = 0; m < 3; ++m) acc[m] += T * ap * c[m];
                T *= 1.0f - ap;
                if (T <= (float)kGenTTerm) break;
            }
            o = make_float4(acc[0], acc[1], acc[2], 1.0f - T);
        }
    }
    out[(size_t)py * G.cam.W + px] = o;
}

// ---------------------------------------------------------------------------
// Image quality of a rendering against a reference (Section 6: SSIM and
// PSNR of VDI renderings against DVR).  RGB of RGBA float32 images, data
// range 1.  SSIM (Wang et al. 2004): 11 x 11 Gaussian window, sigma 1.5,
// K1 = 0.01, K2 = 0.03, population moments, averaged over the pixels whose
// window lies inside the image and over the three channels.  PSNR from the
// mean squared error over all pixels and channels.
// ---------------------------------------------------------------------------
constexpr int kSsimR = 5;                 // window radius
constexpr int kQualityBlock = 256;        // threads per block of the partial-sum kernel

struct SsimWeights {
    double w[2 * kSsimR + 1];             // 1-d Gaussian, normalised to sum 1
};

// Per block: the sum of the SSIM (3 channels summed) of its valid pixels and
// the sum of squared RGB differences of all its pixels, in a fixed order.
__global__ __launch_bounds__(kQualityBlock) void k_quality_partials(const float4 *__restrict__ a,
                                                                    const float4 *__restrict__ b, int W, int H,
                                                                    SsimWeights g, double2 *__restrict__ part)
{
    __shared__ double sh[2][kQualityBlock];
    const size_t n = (size_t)W * H;
    const size_t i = (size_t)blockIdx.x * kQualityBlock + threadIdx.x;
    double ssim = 0.0, se = 0.0;
    if (i < n) {
        const int x = (int)(i % W), y = (int)(i / W);
        const float4 pa = a[i], pb = b[i];
        const double d0 = (double)pa.x - pb.x, d1 = (double)pa.y - pb.y, d2 = (double)pa.z - pb.z;
        se = d0 * d0 + d1 * d1 + d2 * d2;
        if (x >= kSsimR && x < W - kSsimR && y >= kSsimR && y < H - kSsimR) {
            double mx[3] = {0, 0, 0}, my[3] = {0, 0, 0}, sxx[3] = {0, 0, 0}, syy[3] = {0, 0, 0}, sxy[3] = {0, 0, 0};
            for (int dy = -kSsimR; dy <= kSsimR; ++dy)
                for (int dx = -kSsimR; dx <= kSsimR; ++dx) {
                    const double w = g.w[dy + kSsimR] * g.w[dx + kSsimR];
                    const size_t j = (size_t)(y + dy) * W + (x + dx);
                    const float4 qa = a[j], qb = b[j];
                    const double va[3] = {qa.x, qa.y, qa.z}, vb[3] = {qb.x, qb.y, qb.z};
                    for (int c = 0; c < 3; ++c) {
                        mx[c] += w * va[c];
                        my[c] += w * vb[c];
                        sxx[c] += w * va[c] * va[c];
                        syy[c] += w * vb[c] * vb[c];
                        sxy[c] += w * va[c] * vb[c];
                    }
                }
            const double C1 = 0.01 * 0.01, C2 = 0.03 * 0.03;
            for (int c = 0; c < 3; ++c) {
                const double vx = sxx[c] - mx[c] * mx[c], vy = syy[c] - my[c] * my[c];
                const double cxy = sxy[c] - mx[c] * my[c];
                ssim += ((2 * mx[c] * my[c] + C1) * (2 * cxy + C2)) /
                        ((mx[c] * mx[c] + my[c] * my[c] + C1) * (vx + vy + C2));
            }
        }
    }
    sh[0][threadIdx.x] = ssim;
    sh[1][threadIdx.x] = se;
    __syncthreads();
    for (int s = kQualityBlock / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) {
            sh[0][threadIdx.x] += sh[0][threadIdx.x + s];
            sh[1][threadIdx.x] += sh[1][threadIdx.x + s];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = make_double2(sh[0][0], sh[1][0]);
}

// One block sums the partials in a fixed order.
__global__ __launch_bounds__(kQualityBlock) void k_quality_sum(const double2 *__restrict__ part, int nparts,
                                                               double2 *__restrict__ total)
{
    __shared__ double sh[2][kQualityBlock];
    double s0 = 0.0, s1 = 0.0;
    for (int k = threadIdx.x; k < nparts; k += kQualityBlock) {
        s0 += part[k].x;
        s1 += part[k].y;
    }
    sh[0][threadIdx.x] = s0;
    sh[1][threadIdx.x] = s1;
    __syncthreads();
    for (int s = kQualityBlock / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) {
            sh[0][threadIdx.x] += sh[0][threadIdx.x + s];
            sh[1][threadIdx.x] += sh[1][threadIdx.x + s];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) *total = make_double2(sh[0][0], sh[1][0]);
}

void gnorm(double *v)
{
    const double n = sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
    v[0] /= n;
    v[1] /= n;
    v[2] /= n;
}

void gcross(const double *a, const double *b, double *o)
{
    o[0] = a[1] * b[2] - a[2] * b[1];
    o[1] = a[2] * b[0] - a[0] * b[2];
    o[2] = a[0] * b[1] - a[1] * b[0];
}

}  // namespace
}  // namespace vdi

namespace vdi {
namespace {

// Check the arguments and fill the per-call constants of the kernel.
int make_gen_params(const vdi_volume *vol, const vdi_gen_params *p, GenParams &G)
{
    if (!vol || !p || !vol->data) return set_error(VDI_ERR_ARG, "null argument");
    if (vol->nx < 1 || vol->ny < 1 || vol->nz < 1 || vol->nx > 16384 || vol->ny > 16384 || vol->nz > 16384)
        return set_error(VDI_ERR_ARG, "volume size out of range");
    if (vol->voxel_fmt != VDI_VOXEL_F32 && vol->voxel_fmt != VDI_VOXEL_U16)
        return set_error(VDI_ERR_ARG, "unknown voxel format");
    for (int a = 0; a < 3; ++a)
        if (!isfinite(vol->aabb_min[a]) || !isfinite(vol->aabb_max[a]) || !(vol->aabb_max[a] > vol->aabb_min[a]))
            return set_error(VDI_ERR_ARG, "the AABB must be finite and non-empty");
    if (p->width < 1 || p->height < 1 || p->width > 32768 || p->height > 32768)
        return set_error(VDI_ERR_ARG, "VDI size out of range");
    if (p->max_supersegments < 1 || p->max_supersegments > VDI_MAX_SUPERSEGMENTS)
        return set_error(VDI_ERR_ARG, "max_supersegments must be in [1, 255]");
    if (p->tf != VDI_TF_RAMP && p->tf != VDI_TF_KNOTS4) return set_error(VDI_ERR_ARG, "unknown transfer function");
    if (!isfinite(p->gamma) || p->gamma < 0.0) return set_error(VDI_ERR_ARG, "gamma must be finite and >= 0");
    const vdi_camera &c = p->camera_VO;
    const float cv[11] = {c.eye[0], c.eye[1], c.eye[2], c.target[0], c.target[1], c.target[2],
                          c.up[0],  c.up[1],  c.up[2],  c.fov_y_deg, c.near_plane};
    for (float x : cv)
        if (!isfinite(x)) return set_error(VDI_ERR_ARG, "camera has a non-finite value");
    if (!(c.fov_y_deg > 0.0f && c.fov_y_deg < 180.0f) || !(c.near_plane > 0.0f))
        return set_error(VDI_ERR_ARG, "camera fov or near plane out of range");

    memset(&G, 0, sizeof G);
    // V_O basis: F = normalize(target - eye), R = normalize(F x up), U = R x F.
    double up[3];
    for (int a = 0; a < 3; ++a) {
        G.cam.eye[a] = c.eye[a];
        G.cam.F[a] = (double)c.target[a] - (double)c.eye[a];
        up[a] = c.up[a];
    }
    gnorm(G.cam.F);
    gcross(G.cam.F, up, G.cam.R);
    gnorm(G.cam.R);
    gcross(G.cam.R, G.cam.F, G.cam.U);
    for (int a = 0; a < 3; ++a)
        if (!isfinite(G.cam.F[a]) || !isfinite(G.cam.R[a]))
            return set_error(VDI_ERR_ARG, "degenerate camera (target equals eye, or up parallel to the view)");
    G.cam.tanh_ = tan((double)c.fov_y_deg * M_PI / 360.0);
    G.cam.aspect = (double)p->width / (double)p->height;
    G.cam.near_ = c.near_plane;
    G.cam.W = p->width;
    G.cam.H = p->height;
    G.vol.nx = vol->nx;
    G.vol.ny = vol->ny;
    G.vol.nz = vol->nz;
    G.vol.is_u16 = vol->voxel_fmt == VDI_VOXEL_U16;
    G.vol.data = vol->data;
    double ext = 0.0;
    for (int a = 0; a < 3; ++a) {
        G.vol.bmin[a] = vol->aabb_min[a];
        G.vol.bmax[a] = vol->aabb_max[a];
        ext = std::max(ext, vol->aabb_max[a] - vol->aabb_min[a]);
    }
    const int nmax = std::max(vol->nx, std::max(vol->ny, vol->nz));
    G.ds = ext / nmax;  // one voxel of the longest axis
    G.maxs = 2 * nmax + 8;
    G.NS = p->max_supersegments;
    G.delta = (int)floor(0.15 * G.NS);
    G.tf = p->tf;
    G.gamma = p->gamma;
    return VDI_OK;
}

}  // namespace
}  // namespace vdi

extern "C" int vdi_generate(const vdi_volume *vol, const vdi_gen_params *p, uint8_t *count, float *depth, float *rgba,
                            double *gamma_out, void *stream)
{
    if (!count || !depth || !rgba) return vdi::set_error(VDI_ERR_ARG, "null output");
    vdi::GenParams G;
    const int rc = vdi::make_gen_params(vol, p, G);
    if (rc) return rc;
    hipStream_t st = static_cast<hipStream_t>(stream);
    // Persistent grid: as many single-wavefront workgroups as fit on the device at once.
    int device = 0, cus = 0, per_cu = 0;
    hipError_t e = hipGetDevice(&device);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device);
    if (e == hipSuccess) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, vdi::k_generate, 64, 0);
    if (e != hipSuccess) return vdi::hip_error(e, "device query");
    const long long ntiles = (long long)((p->width + vdi::kGenTileW - 1) / vdi::kGenTileW) *
                             ((p->height + vdi::kGenTileH - 1) / vdi::kGenTileH);
    const int blocks = (int)std::max<long long>(1, std::min<long long>(ntiles, (long long)std::max(1, cus * per_cu)));
    // Each lane caches up to K samples: all of them (2 max(n) + 8) while the cache fits the budget.
    const int K = (int)std::min<size_t>((size_t)G.maxs, vdi::kGenCacheBytes / ((size_t)blocks * 64 * sizeof(double2)));
    const size_t cache_bytes = (size_t)blocks * K * 64 * sizeof(double2);
    size_t bytes = (size_t)1 << 20;
    while (bytes < 256 + cache_bytes) bytes <<= 1;
    hipMemPool_t pool = nullptr;
    e = vdi::library_pool(device, &pool);
    if (e != hipSuccess) return vdi::hip_error(e, "scratch pool");
    char *scratch = nullptr;
    e = hipMallocFromPoolAsync((void **)&scratch, bytes, pool, st);
    if (e != hipSuccess) return vdi::set_error(VDI_ERR_OOM, "generation scratch (%zu bytes)", bytes);
    e = hipMemsetAsync(scratch, 0, sizeof(unsigned), st);
    if (e == hipSuccess) {
        vdi::k_generate<<<blocks, 64, 0, st>>>(G, reinterpret_cast<unsigned *>(scratch), (int)ntiles,
                                               reinterpret_cast<double2 *>(scratch + 256), K, count,
                                               reinterpret_cast<float2 *>(depth), reinterpret_cast<float4 *>(rgba),
                                               gamma_out);
        e = hipGetLastError();
    }
    const hipError_t e2 = hipFreeAsync(scratch, st);
    if (e == hipSuccess) e = e2;
    if (e != hipSuccess) return vdi::hip_error(e, "generation launch");
    return VDI_OK;
}

extern "C" int vdi_dvr(const vdi_volume *vol, const vdi_dvr_params *p, float *out_rgba, void *stream)
{
    if (!p || !out_rgba) return vdi::set_error(VDI_ERR_ARG, "null argument");
    if (p->precision != VDI_DVR_F64 && p->precision != VDI_DVR_F32)
        return vdi::set_error(VDI_ERR_ARG, "unknown DVR precision");
    if (p->width > 16384 || p->height > 16384) return vdi::set_error(VDI_ERR_ARG, "image size out of range");
    vdi_gen_params gp;
    memset(&gp, 0, sizeof gp);
    gp.camera_VO = p->camera;
    gp.width = p->width;
    gp.height = p->height;
    gp.max_supersegments = 1;
    gp.tf = p->tf;
    vdi::GenParams G;
    const int rc = vdi::make_gen_params(vol, &gp, G);
    if (rc) return rc;
    const dim3 grid((unsigned)((p->width + 63) / 64), (unsigned)p->height);
    auto *out = reinterpret_cast<float4 *>(out_rgba);
    if (p->precision == VDI_DVR_F64)
        vdi::k_dvr<true><<<grid, 64, 0, static_cast<hipStream_t>(stream)>>>(G, out);
    else
        vdi::k_dvr<false><<<grid, 64, 0, static_cast<hipStream_t>(stream)>>>(G, out);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return vdi::hip_error(e, "DVR launch");
    return VDI_OK;
}

extern "C" int vdi_image_quality(const float *image, const float *reference, int32_t width, int32_t height,
                                 double *ssim, double *psnr, void *stream)
{
    if (!image || !reference || !ssim || !psnr) return vdi::set_error(VDI_ERR_ARG, "null argument");
    if (width < 2 * vdi::kSsimR + 1 || height < 2 * vdi::kSsimR + 1 || width > 16384 || height > 16384)
        return vdi::set_error(VDI_ERR_ARG, "images must be 11x11 to 16384x16384 (the SSIM window is 11x11)");
    vdi::SsimWeights g;
    double sum = 0.0;
    for (int k = -vdi::kSsimR; k <= vdi::kSsimR; ++k) sum += (g.w[k + vdi::kSsimR] = exp(-(k * k) / (2.0 * 1.5 * 1.5)));
    for (double &w : g.w) w /= sum;
    const size_t n = (size_t)width * height;
    const int nparts = (int)((n + vdi::kQualityBlock - 1) / vdi::kQualityBlock);
    hipStream_t st = static_cast<hipStream_t>(stream);
    double2 *d_part = nullptr;
    hipError_t e = hipMallocAsync((void **)&d_part, (nparts + 1) * sizeof(double2), st);
    if (e != hipSuccess) return vdi::hip_error(e, "quality scratch");
    vdi::k_quality_partials<<<nparts, vdi::kQualityBlock, 0, st>>>(reinterpret_cast<const float4 *>(image),
                                                                   reinterpret_cast<const float4 *>(reference), width,
                                                                   height, g, d_part);
    vdi::k_quality_sum<<<1, vdi::kQualityBlock, 0, st>>>(d_part, nparts, d_part + nparts);
    double2 tot = make_double2(0.0, 0.0);
    e = hipGetLastError();
    if (e == hipSuccess) e = hipMemcpyAsync(&tot, d_part + nparts, sizeof tot, hipMemcpyDeviceToHost, st);
    const hipError_t e2 = hipFreeAsync(d_part, st);
    if (e == hipSuccess) e = e2;
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return vdi::hip_error(e, "quality");
    const double valid = (double)(width - 2 * vdi::kSsimR) * (height - 2 * vdi::kSsimR) * 3.0;
    *ssim = tot.x / valid;
    const double mse = tot.y / (3.0 * (double)n);
    *psnr = mse > 0.0 ? 10.0 * log10(1.0 / mse) : INFINITY;
    return VDI_OK;
}
