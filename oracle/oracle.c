/*
 * FP64 reference renderer for Volumetric Depth Images.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this library.  It shares no code,
 * header, table or helper with the HIP renderer; the two meet only in the
 * seeded input arrays.
 *
 * What it computes (plain definitions, written for checking by eye):
 *
 *  Exact mode.  The VDI defines a piecewise-constant emission-absorption
 *  field: supersegment S_ij occupies the points whose V_O NDC position lies in
 *  list i's pixel cell (lists form a regular grid of 2/w x 2/h cells in NDC,
 *  Section 4.1 / Fig. 3) and whose V_O view depth lies in [f_ij, b_ij]
 *  (Section 2.3).  A V_N pixel ray is clipped to the AABB and the V_O frustum
 *  (Section 4.1), cut at every list-grid line it crosses, each piece is
 *  overlapped with every supersegment of its list (linear scan), the pieces
 *  are ordered along the ray, and each contributes opacity corrected for its
 *  length by Eq. 2 with exponent l = (world length) / (world length of the
 *  generating ray inside S_ij), composited front to back with early ray
 *  termination at transmittance 1e-5.
 *
 *  Preview mode (Section 4.4).  The ray walks the cells of the count grid
 *  (Section 4.3); a non-empty cell crossed over [ua,ub] receives
 *  n = ceil(((ub-ua)/slice depth) * (count / k^2) / D_R) samples at regular
 *  spacing h; each sample looks up the supersegment containing it (half-open
 *  [f, b)) and contributes opacity corrected with exponent h / L0.  Pixels
 *  whose result hinges on a floating-point tie (a sample within 1e-6 pixel of
 *  a list edge, within 1e-7 relative of a supersegment face, or a ceil
 *  argument within 1e-7 relative of an integer) are flagged.
 *
 *  Image downsampling renders round(W/D_I) x round(H/D_I) rays with
 *  the same camera and upsamples bilinearly (half-pixel centres, clamped).
 *
 *  Count grid (Section 4.3): for each k x k block of lists and each depth
 *  slice [Z_c, Z_c+1), the number of supersegments of those lists with
 *  f < Z_c+1 and b > Z_c.
 *
 *  Brute-force marcher: midpoint rule with M steps over the clipped ray, each
 *  step taking the supersegment whose closed depth interval holds the point.
 *
 * Build: gcc -O2 -fopenmp -shared -fPIC (driven by oracle/__init__.py).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define T_TERM 1e-5

typedef struct {
    int32_t W, H, NS;
    int32_t grid_k, grid_nz;
    const float *cam;     /* V_O: eye[3] target[3] up[3] fov_y_deg near */
    const double *bmin;   /* [3] */
    const double *bmax;   /* [3] */
    const uint8_t *count; /* [H][W] */
    const float *depth;   /* [NS][H][W][2] */
    const float *rgba;    /* [NS][H][W][4] straight colour, opacity */
    const float *grid_z;  /* [grid_nz+1] */
    const uint32_t *grid; /* [grid_nz][GH][GW], may be NULL for exact mode */
} or_vdi_t;

typedef struct {
    double eye[3], F[3], R[3], U[3];
    double th, aspect, near_;
    int W, H;
} ocam_t;

static double dot3(const double *a, const double *b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }

static void unit3(double *v)
{
    double n = sqrt(dot3(v, v));
    v[0] /= n; v[1] /= n; v[2] /= n;
}

static void cross3(const double *a, const double *b, double *o)
{
    o[0] = a[1] * b[2] - a[2] * b[1];
    o[1] = a[2] * b[0] - a[0] * b[2];
    o[2] = a[0] * b[1] - a[1] * b[0];
}

/* aspect <= 0: W / H. */
static void ocam_init(ocam_t *c, const float *cam, int W, int H, double aspect)
{
    double up[3];
    for (int a = 0; a < 3; ++a) {
        c->eye[a] = cam[a];
        c->F[a] = (double)cam[3 + a] - (double)cam[a];
        up[a] = cam[6 + a];
    }
    unit3(c->F);
    cross3(c->F, up, c->R);
    unit3(c->R);
    cross3(c->R, c->F, c->U);
    c->th = tan((double)cam[9] * M_PI / 360.0);
    c->aspect = aspect > 0.0 ? aspect : (double)W / (double)H;
    c->near_ = cam[10];
    c->W = W;
    c->H = H;
}

/* Unit direction through NDC point (xc, yc) of camera c. */
static void ocam_dir(const ocam_t *c, double xc, double yc, double *d)
{
    for (int a = 0; a < 3; ++a) d[a] = c->F[a] + xc * c->th * c->aspect * c->R[a] + yc * c->th * c->U[a];
    unit3(d);
}

/* A V_N ray expressed in V_O's frame: X(t) = X0 + t Xp (scaled so that
 * x_ndc = X/Z), Y likewise, Z(t) = Z0 + t Zp is V_O view depth. */
typedef struct {
    double X0, Xp, Y0, Yp, Z0, Zp;
    double t0, t1;
} oray_t;

static int clip_half(double a, double b, double *lo, double *hi)
{
    /* keep t with a + b t >= 0 */
    if (b == 0.0) return a >= 0.0;
    double t = -a / b;
    if (b > 0.0) { if (t > *lo) *lo = t; }
    else { if (t < *hi) *hi = t; }
    return 1;
}

/* Returns 1 and fills r if the clipped ray is non-empty. */
static int oray_setup(const or_vdi_t *v, const ocam_t *cO, const ocam_t *cN, double xc, double yc, oray_t *r)
{
    double d[3], e[3], rel[3];
    ocam_dir(cN, xc, yc, d);
    for (int a = 0; a < 3; ++a) { e[a] = cN->eye[a]; rel[a] = e[a] - cO->eye[a]; }
    double sx = 1.0 / (cO->th * cO->aspect), sy = 1.0 / cO->th;
    r->X0 = dot3(cO->R, rel) * sx;
    r->Xp = dot3(cO->R, d) * sx;
    r->Y0 = dot3(cO->U, rel) * sy;
    r->Yp = dot3(cO->U, d) * sy;
    r->Z0 = dot3(cO->F, rel);
    r->Zp = dot3(cO->F, d);
    double lo = 0.0, hi = INFINITY;
    /* V_N near plane */
    if (!clip_half(-cN->near_, dot3(cN->F, d), &lo, &hi)) return 0;
    /* AABB */
    for (int a = 0; a < 3; ++a) {
        if (!clip_half(e[a] - v->bmin[a], d[a], &lo, &hi)) return 0;
        if (!clip_half(v->bmax[a] - e[a], -d[a], &lo, &hi)) return 0;
    }
    /* V_O frustum: Z >= near, |X| <= Z, |Y| <= Z */
    if (!clip_half(r->Z0 - cO->near_, r->Zp, &lo, &hi)) return 0;
    if (!clip_half(r->Z0 - r->X0, r->Zp - r->Xp, &lo, &hi)) return 0;
    if (!clip_half(r->Z0 + r->X0, r->Zp + r->Xp, &lo, &hi)) return 0;
    if (!clip_half(r->Z0 - r->Y0, r->Zp - r->Yp, &lo, &hi)) return 0;
    if (!clip_half(r->Z0 + r->Y0, r->Zp + r->Yp, &lo, &hi)) return 0;
    r->t0 = lo;
    r->t1 = hi;
    return hi > lo;
}

static inline double ox(const oray_t *r, double t) { return (r->X0 + t * r->Xp) / (r->Z0 + t * r->Zp); }
static inline double oy(const oray_t *r, double t) { return (r->Y0 + t * r->Yp) / (r->Z0 + t * r->Zp); }
static inline double oz(const oray_t *r, double t) { return r->Z0 + t * r->Zp; }

static int cmp_dbl(const void *a, const void *b)
{
    double x = *(const double *)a, y = *(const double *)b;
    return (x > y) - (x < y);
}

/* Threads of one parallel region: nthreads > 0, else the OpenMP default
 * (set per region, so a one-thread call leaves later calls unchanged). */
static int oracle_threads(int nthreads)
{
#ifdef _OPENMP
    return nthreads > 0 ? nthreads : omp_get_max_threads();
#else
    (void)nthreads;
    return 1;
#endif
}

static inline int clampi(int x, int lo, int hi) { return x < lo ? lo : (x > hi ? hi : x); }

static inline int list_col(const or_vdi_t *v, double xn) { return clampi((int)floor((xn + 1.0) * v->W / 2.0), 0, v->W - 1); }
static inline int list_row(const or_vdi_t *v, double yn) { return clampi((int)floor((yn + 1.0) * v->H / 2.0), 0, v->H - 1); }

/* Append the parameters where the ray crosses NDC lines coord = -1 + 2 m step / n,
 * 0 < m step < n, strictly inside (t0, t1).  axis 0: x, 1: y. */
static int add_crossings(const oray_t *r, int axis, int n, int step, double *ts, int nts)
{
    double a = axis == 0 ? ox(r, r->t0) : oy(r, r->t0);
    double b = axis == 0 ? ox(r, r->t1) : oy(r, r->t1);
    double lo = fmin(a, b), hi = fmax(a, b);
    double P0 = axis == 0 ? r->X0 : r->Y0, Pp = axis == 0 ? r->Xp : r->Yp;
    for (int m = step; m < n; m += step) {
        double c = -1.0 + 2.0 * m / n;
        if (!(c > lo && c < hi)) continue;
        double t = (c * r->Z0 - P0) / (Pp - c * r->Zp);
        if (t > r->t0 && t < r->t1) ts[nts++] = t;
    }
    return nts;
}

/* cos of the angle between list (px,py)'s generating ray and V_O's axis. */
static double list_cos(const or_vdi_t *v, const ocam_t *cO, int px, int py)
{
    double di[3];
    ocam_dir(cO, -1.0 + (2.0 * px + 1.0) / v->W, -1.0 + (2.0 * py + 1.0) / v->H, di);
    return dot3(cO->F, di);
}

typedef struct {
    double tlo, thi, l;
    int32_t list, j;
} piece_t;

static int cmp_piece(const void *a, const void *b)
{
    const piece_t *x = (const piece_t *)a, *y = (const piece_t *)b;
    if (x->tlo != y->tlo) return (x->tlo > y->tlo) - (x->tlo < y->tlo);
    return (x->list > y->list) - (x->list < y->list);
}

/* Eq. 2 with 0^l = 0 for l > 0. */
static double corrected_alpha(double a, double l)
{
    if (a >= 1.0) return 1.0;
    return 1.0 - pow(1.0 - a, l);
}

typedef struct {
    int64_t lists, pieces; /* per pixel: list sub-intervals entered before termination; pieces composited */
    int64_t lists_ess;     /* those of the sub-intervals that lie partly in a non-empty grid cell */
} ostat_t;

/*
 * Exact render of one V_N pixel-centre ray (NDC xc, yc).
 * touched_lists [H*W] / touched_S [NS*H*W] (optional) receive 1 for every list
 * entered before termination and every supersegment composited.
 */
/* Whether the depth range [zlo, zhi] of list li holds any part of a non-empty
 * grid cell (Section 4.3): a slice overlapping it with positive length whose
 * count for li's column is non-zero.  A list sub-interval that fails this
 * holds no supersegment, so empty-space skipping need not read the list. */
static int in_nonempty_cell(const or_vdi_t *v, int px, int py, double zlo, double zhi)
{
    const int k = v->grid_k, GW = (v->W + k - 1) / k, GH = (v->H + k - 1) / k;
    for (int c = 0; c < v->grid_nz; ++c) {
        double s0 = v->grid_z[c], s1 = v->grid_z[c + 1];
        int overlap = zhi > zlo ? (s0 < zhi && s1 > zlo) : (s0 <= zlo && zlo < s1);
        if (overlap && v->grid[((size_t)c * GH + py / k) * GW + px / k] != 0) return 1;
    }
    return 0;
}

/*
 * Ties in exact mode.  A ray that lies in a list-edge plane over a part of its
 * length (e.g. a pixel-centre ray of a downsampled grid seen from V_O itself,
 * which runs along the corner of four lists) has no unique list there: either
 * side is a valid reading of the field.  The list of each sub-interval is
 * located at its midpoint; bx, by in {-1, 0, +1} shift that location by that
 * many BIAS_PX pixel, so every such decision of the ray goes the same way.
 * *flag is set when the ray runs along an edge plane (its list coordinate in
 * x or y varies by at most 2e-6 pixel over the clipped ray) and a
 * sub-interval of positive length has both ends within 1e-6 pixel of an edge.
 */
#define BIAS_PX 1e-9

/* Both ends of a sub-interval within 1e-6 pixel of one list edge. */
static int on_edge(double fa, double fb)
{
    return fabs(fa - nearbyint(fa)) <= 1e-6 && fabs(fb - nearbyint(fb)) <= 1e-6 && nearbyint(fa) == nearbyint(fb);
}

static void exact_pixel(const or_vdi_t *v, const ocam_t *cO, const ocam_t *cN, double xc, double yc, double bx,
                        double by, double *out, uint8_t *flag, ostat_t *st, uint8_t *touched_lists,
                        uint8_t *touched_S, uint8_t *touched_ess, double *ts, piece_t *pc, int32_t *sub_list,
                        double *sub_t, uint8_t *sub_need)
{
    out[0] = out[1] = out[2] = out[3] = 0.0;
    if (flag) *flag = 0;
    if (st) st->lists = st->pieces = st->lists_ess = 0;
    oray_t r;
    if (!oray_setup(v, cO, cN, xc, yc, &r)) return;
    int nts = 0;
    ts[nts++] = r.t0;
    ts[nts++] = r.t1;
    nts = add_crossings(&r, 0, v->W, 1, ts, nts);
    nts = add_crossings(&r, 1, v->H, 1, ts, nts);
    qsort(ts, nts, sizeof(double), cmp_dbl);
    /* The ray runs along a list-edge plane (x or y) when its list coordinate
     * varies by at most 2e-6 pixel over the whole clipped ray. */
    const int along_x = fabs(ox(&r, r.t1) - ox(&r, r.t0)) * v->W / 2.0 <= 2e-6;
    const int along_y = fabs(oy(&r, r.t1) - oy(&r, r.t0)) * v->H / 2.0 <= 2e-6;
    const size_t plane = (size_t)v->W * v->H;
    int np = 0, nsub = 0;
    const int zflat = fabs(r.Zp) < 1e-12;
    for (int s = 0; s + 1 < nts; ++s) {
        double ta = ts[s], tb = ts[s + 1];
        if (!(tb > ta)) continue;
        double tm = 0.5 * (ta + tb);
        if (flag && ((along_x && on_edge((ox(&r, ta) + 1.0) * v->W / 2.0, (ox(&r, tb) + 1.0) * v->W / 2.0)) ||
                     (along_y && on_edge((oy(&r, ta) + 1.0) * v->H / 2.0, (oy(&r, tb) + 1.0) * v->H / 2.0))))
            *flag = 1;
        int px = clampi((int)floor((ox(&r, tm) + 1.0) * v->W / 2.0 + bx * BIAS_PX), 0, v->W - 1);
        int py = clampi((int)floor((oy(&r, tm) + 1.0) * v->H / 2.0 + by * BIAS_PX), 0, v->H - 1);
        int li = py * v->W + px;
        double za = oz(&r, ta), zb = oz(&r, tb);
        sub_list[nsub] = li;
        sub_t[nsub] = ta;
        sub_need[nsub] = touched_ess ? (uint8_t)in_nonempty_cell(v, px, py, fmin(za, zb), fmax(za, zb)) : 0;
        ++nsub;
        int n = v->count[li];
        if (n == 0) continue;
        double cth = list_cos(v, cO, px, py);
        for (int j = 0; j < n; ++j) {
            size_t o = (size_t)j * plane + li;
            double f = v->depth[2 * o], b = v->depth[2 * o + 1];
            double tlo, thi, L;
            if (zflat) {
                if (!(f <= za && za < b)) continue;
                tlo = ta;
                thi = tb;
                L = tb - ta;
            } else {
                double zlo = fmax(fmin(za, zb), f), zhi = fmin(fmax(za, zb), b);
                if (!(zhi > zlo)) continue;
                double u1 = (zlo - r.Z0) / r.Zp, u2 = (zhi - r.Z0) / r.Zp;
                tlo = fmin(u1, u2);
                thi = fmax(u1, u2);
                L = (zhi - zlo) / fabs(r.Zp);
            }
            double L0 = (b - f) / cth;
            pc[np].tlo = tlo;
            pc[np].thi = thi;
            pc[np].l = L / L0;
            pc[np].list = li;
            pc[np].j = j;
            ++np;
        }
    }
    qsort(pc, np, sizeof(piece_t), cmp_piece);
    double T = 1.0, C[3] = {0, 0, 0}, tstop = r.t1;
    int used = 0;
    for (int k = 0; k < np; ++k) {
        if (!(pc[k].l > 0.0)) continue;
        size_t o = (size_t)pc[k].j * plane + pc[k].list;
        const float *c = v->rgba + 4 * o;
        double at = corrected_alpha(c[3], pc[k].l);
        for (int m = 0; m < 3; ++m) C[m] += T * at * c[m];
        T *= 1.0 - at;
        ++used;
        if (touched_S) touched_S[o] = 1;
        if (T <= T_TERM) { tstop = pc[k].thi; break; }
    }
    out[0] = C[0]; out[1] = C[1]; out[2] = C[2]; out[3] = 1.0 - T;
    int64_t nl = 0, ne = 0;
    for (int s = 0; s < nsub; ++s)
        if (sub_t[s] < tstop) {
            ++nl;
            if (touched_lists) touched_lists[sub_list[s]] = 1;
            if (touched_ess && sub_need[s]) {
                touched_ess[sub_list[s]] = 1;
                ++ne;
            }
        }
    if (st) { st->lists = nl; st->pieces = used; st->lists_ess = ne; }
}

static int max_breaks(const or_vdi_t *v) { return v->W + v->H + v->grid_nz + 8; }

/*
 * Exact render.  aspect <= 0 means W/H (a downsampled render passes the
 * display's).  If pix is NULL, renders all W*H pixels of V_N (row-major,
 * row 0 = bottom) into out[H*W*4]; else renders the npix pixel indices
 * (py*W + px) into out[npix*4].  stats (optional) [npix or W*H][3] = lists,
 * pieces, lists in non-empty grid cells (the last only with touched_ess).
 * touched_ess (optional, needs v->grid) marks the lists entered before
 * termination over a sub-interval that lies partly in a non-empty grid cell.
 */
int or_render_exact(const or_vdi_t *v, const float *camN, int W, int H, double aspect, int64_t npix,
                    const int64_t *pix, double *out, int64_t *stats, uint8_t *touched_lists, uint8_t *touched_S,
                    uint8_t *touched_ess, uint8_t *flags, const double *bias, int nthreads)
{
    if (touched_ess && !v->grid) return -1;
    ocam_t cO, cN;
    ocam_init(&cO, v->cam, v->W, v->H, 0.0);
    ocam_init(&cN, camN, W, H, aspect);
    if (!pix) npix = (int64_t)W * H;
    int nb = max_breaks(v);
    int maxp = nb * (v->NS + 1);
#pragma omp parallel num_threads(oracle_threads(nthreads))
    {
        double *ts = (double *)malloc(sizeof(double) * nb);
        piece_t *pc = (piece_t *)malloc(sizeof(piece_t) * maxp);
        int32_t *sl = (int32_t *)malloc(sizeof(int32_t) * nb);
        double *stt = (double *)malloc(sizeof(double) * nb);
        uint8_t *need = (uint8_t *)malloc(nb);
#pragma omp for schedule(dynamic, 64)
        for (int64_t k = 0; k < npix; ++k) {
            int64_t id = pix ? pix[k] : k;
            int px = (int)(id % W), py = (int)(id / W);
            ostat_t st;
            exact_pixel(v, &cO, &cN, -1.0 + (2.0 * px + 1.0) / W, -1.0 + (2.0 * py + 1.0) / H,
                        bias ? bias[0] : 0.0, bias ? bias[1] : 0.0, out + 4 * k, flags ? flags + k : NULL, &st,
                        touched_lists, touched_S, touched_ess, ts, pc, sl, stt, need);
            if (stats) { stats[3 * k] = st.lists; stats[3 * k + 1] = st.pieces; stats[3 * k + 2] = st.lists_ess; }
        }
        free(ts); free(pc); free(sl); free(stt); free(need);
    }
    return 0;
}

/* ------------------------------------------------------------------ */
/* Preview (Section 4.4)                                                */
/* ------------------------------------------------------------------ */
static inline int near_int(double x, double tol) { return fabs(x - nearbyint(x)) <= tol; }

/*
 * Tie resolution.  A point sample that lies exactly on a list edge or a
 * supersegment face, or a sample count whose ceil argument is an integer, is
 * decided by rounding and may land on either side.  bias (optional, NULL =
 * none) moves every such decision of the ray the same way: bias[0] and
 * bias[1] in {-1, 0, +1} shift the sample's list coordinates by that many
 * 1e-9 pixel in x and y, bias[2] its depth by that many 1e-11 relative before
 * the face tests, bias[3] each ceil argument by that many 1e-10 relative.
 * These shifts are far above FP64 rounding and far below the flag tolerances
 * (1e-6 pixel, 1e-7 relative), so they change only flagged decisions; the
 * flags are taken on the unshifted values.
 */
#define BIAS_Z 1e-11
#define BIAS_N 1e-10

static void preview_pixel(const or_vdi_t *v, const ocam_t *cO, const ocam_t *cN, double xc, double yc, double DR,
                          const double *bias, double *out, uint8_t *flag, int64_t *nsamples, double *ts)
{
    const double bx = bias ? bias[0] : 0.0, by = bias ? bias[1] : 0.0;
    const double bz = bias ? bias[2] : 0.0, bn = bias ? bias[3] : 0.0;
    out[0] = out[1] = out[2] = out[3] = 0.0;
    *flag = 0;
    *nsamples = 0;
    oray_t r;
    if (!oray_setup(v, cO, cN, xc, yc, &r)) return;
    const int k = v->grid_k, GW = (v->W + k - 1) / k, GH = (v->H + k - 1) / k;
    int nts = 0;
    ts[nts++] = r.t0;
    ts[nts++] = r.t1;
    nts = add_crossings(&r, 0, v->W, k, ts, nts);
    nts = add_crossings(&r, 1, v->H, k, ts, nts);
    if (fabs(r.Zp) >= 1e-12)
        for (int c = 0; c <= v->grid_nz; ++c) {
            double t = ((double)v->grid_z[c] - r.Z0) / r.Zp;
            if (t > r.t0 && t < r.t1) ts[nts++] = t;
        }
    qsort(ts, nts, sizeof(double), cmp_dbl);
    const size_t plane = (size_t)v->W * v->H;
    double T = 1.0, C[3] = {0, 0, 0};
    for (int s = 0; s + 1 < nts; ++s) {
        double ua = ts[s], ub = ts[s + 1];
        if (!(ub > ua)) continue;
        double um = 0.5 * (ua + ub);
        int cx = list_col(v, ox(&r, um)) / k, cy = list_row(v, oy(&r, um)) / k;
        double zm = oz(&r, um);
        int cz = 0;
        while (cz + 1 < v->grid_nz && (double)v->grid_z[cz + 1] <= zm) ++cz;
        uint32_t G = v->grid[((size_t)cz * GH + cy) * GW + cx];
        if (G == 0) continue;
        double dz = (double)v->grid_z[cz + 1] - (double)v->grid_z[cz];
        double x = ((ub - ua) / dz) * ((double)G / (double)(k * k)) / DR;
        if (near_int(x, 1e-7 * fmax(1.0, x))) *flag = 1;
        int64_t n = (int64_t)ceil(x + bn * BIAS_N * fmax(1.0, x));
        if (n < 1) n = 1;
        double h = (ub - ua) / (double)n;
        for (int64_t q = 0; q < n; ++q) {
            double u = ua + (q + 0.5) * h;
            double xn = ox(&r, u), yn = oy(&r, u), z = oz(&r, u);
            double fx = (xn + 1.0) * v->W / 2.0, fy = (yn + 1.0) * v->H / 2.0;
            if (near_int(fx, 1e-6) || near_int(fy, 1e-6)) *flag = 1;
            int px = clampi((int)floor(fx + bx * BIAS_PX), 0, v->W - 1);
            int py = clampi((int)floor(fy + by * BIAS_PX), 0, v->H - 1);
            double zs = z + bz * BIAS_Z * z;
            int li = py * v->W + px;
            int nl = v->count[li];
            ++*nsamples;
            for (int j = 0; j < nl; ++j) {
                size_t o = (size_t)j * plane + li;
                double f = v->depth[2 * o], b = v->depth[2 * o + 1];
                if (fabs(z - f) <= 1e-7 * z || fabs(z - b) <= 1e-7 * z) *flag = 1;
                if (f <= zs && zs < b) {
                    const float *c = v->rgba + 4 * o;
                    double L0 = (b - f) / list_cos(v, cO, px, py);
                    double at = corrected_alpha(c[3], h / L0);
                    for (int m = 0; m < 3; ++m) C[m] += T * at * c[m];
                    T *= 1.0 - at;
                    break;
                }
            }
            if (T <= T_TERM) goto done;
        }
    }
done:
    out[0] = C[0]; out[1] = C[1]; out[2] = C[2]; out[3] = 1.0 - T;
}

/*
 * Along-ray subsampled render (D_R > 0) of a w x h image with V_N's camera
 * (aspect <= 0: w/h; a downsampled render passes the display's W/H).  pix / npix as in or_render_exact.  flags[npix] receive the
 * tie flags; nsamp[npix] (optional) the number of point samples taken; bias
 * (optional, 4 values) resolves ties one way (see preview_pixel).
 */
int or_render_preview(const or_vdi_t *v, const float *camN, int w, int h, double aspect, double DR, int64_t npix,
                      const int64_t *pix, double *out, uint8_t *flags, int64_t *nsamp, const double *bias, int nthreads)
{
    if (!(DR > 0.0) || !v->grid) return -1;
    ocam_t cO, cN;
    ocam_init(&cO, v->cam, v->W, v->H, 0.0);
    ocam_init(&cN, camN, w, h, aspect);
    if (!pix) npix = (int64_t)w * h;
    int nb = max_breaks(v);
#pragma omp parallel num_threads(oracle_threads(nthreads))
    {
        double *ts = (double *)malloc(sizeof(double) * nb);
#pragma omp for schedule(dynamic, 16)
        for (int64_t q = 0; q < npix; ++q) {
            int64_t id = pix ? pix[q] : q;
            int px = (int)(id % w), py = (int)(id / w);
            int64_t ns;
            preview_pixel(v, &cO, &cN, -1.0 + (2.0 * px + 1.0) / w, -1.0 + (2.0 * py + 1.0) / h, DR, bias,
                          out + 4 * q, flags + q, &ns, ts);
            if (nsamp) nsamp[q] = ns;
        }
        free(ts);
    }
    return 0;
}

/*
 * Bilinear upsampling of lo[h][w][4] to out[H][W][4] with half-pixel centres,
 * clamped at the edges.  lo_flags (optional) propagate to out_flags: an output
 * pixel is flagged if any of its four source texels is.
 */
void or_upsample(const double *lo, const uint8_t *lo_flags, int w, int h, int W, int H, double *out, uint8_t *out_flags)
{
    for (int y = 0; y < H; ++y)
        for (int x = 0; x < W; ++x) {
            double sx = (x + 0.5) * (double)w / W - 0.5, sy = (y + 0.5) * (double)h / H - 0.5;
            if (sx < 0.0) sx = 0.0;
            if (sy < 0.0) sy = 0.0;
            if (sx > w - 1) sx = w - 1;
            if (sy > h - 1) sy = h - 1;
            int x0 = (int)floor(sx), y0 = (int)floor(sy);
            int x1 = x0 + 1 < w ? x0 + 1 : w - 1, y1 = y0 + 1 < h ? y0 + 1 : h - 1;
            double fx = sx - x0, fy = sy - y0;
            for (int m = 0; m < 4; ++m) {
                double a = lo[4 * ((size_t)y0 * w + x0) + m], b = lo[4 * ((size_t)y0 * w + x1) + m];
                double c = lo[4 * ((size_t)y1 * w + x0) + m], d = lo[4 * ((size_t)y1 * w + x1) + m];
                out[4 * ((size_t)y * W + x) + m] = (a * (1 - fx) + b * fx) * (1 - fy) + (c * (1 - fx) + d * fx) * fy;
            }
            if (out_flags)
                out_flags[(size_t)y * W + x] = lo_flags ? (lo_flags[(size_t)y0 * w + x0] | lo_flags[(size_t)y0 * w + x1] |
                                                           lo_flags[(size_t)y1 * w + x0] | lo_flags[(size_t)y1 * w + x1])
                                                        : 0;
        }
}

/* Count grid (Section 4.3): out[grid_nz][GH][GW]. */
void or_count_grid(const or_vdi_t *v, uint32_t *out)
{
    const int k = v->grid_k, GW = (v->W + k - 1) / k, GH = (v->H + k - 1) / k;
    memset(out, 0, sizeof(uint32_t) * (size_t)v->grid_nz * GH * GW);
    const size_t plane = (size_t)v->W * v->H;
    for (int py = 0; py < v->H; ++py)
        for (int px = 0; px < v->W; ++px) {
            int li = py * v->W + px, n = v->count[li];
            for (int j = 0; j < n; ++j) {
                size_t o = (size_t)j * plane + li;
                float f = v->depth[2 * o], b = v->depth[2 * o + 1];
                for (int c = 0; c < v->grid_nz; ++c)
                    if (f < v->grid_z[c + 1] && b > v->grid_z[c]) ++out[((size_t)c * GH + py / k) * GW + px / k];
            }
        }
}

/* Brute-force midpoint marching of the piecewise-constant field, M steps. */
int or_march(const or_vdi_t *v, const float *camN, int W, int H, int64_t npix, const int64_t *pix, int64_t M,
             double *out, int nthreads)
{
    ocam_t cO, cN;
    ocam_init(&cO, v->cam, v->W, v->H, 0.0);
    ocam_init(&cN, camN, W, H, 0.0);
    const size_t plane = (size_t)v->W * v->H;
#pragma omp parallel for schedule(dynamic, 1) num_threads(oracle_threads(nthreads))
    for (int64_t q = 0; q < npix; ++q) {
        int64_t id = pix[q];
        int px = (int)(id % W), py = (int)(id / W);
        double *o4 = out + 4 * q;
        o4[0] = o4[1] = o4[2] = o4[3] = 0.0;
        oray_t r;
        if (!oray_setup(v, &cO, &cN, -1.0 + (2.0 * px + 1.0) / W, -1.0 + (2.0 * py + 1.0) / H, &r)) continue;
        double h = (r.t1 - r.t0) / (double)M, T = 1.0, C[3] = {0, 0, 0};
        for (int64_t s = 0; s < M; ++s) {
            double u = r.t0 + (s + 0.5) * h;
            int lx = list_col(v, ox(&r, u)), ly = list_row(v, oy(&r, u));
            int li = ly * v->W + lx;
            double z = oz(&r, u);
            for (int j = 0; j < v->count[li]; ++j) {
                size_t o = (size_t)j * plane + li;
                double f = v->depth[2 * o], b = v->depth[2 * o + 1];
                if (f <= z && z <= b) {
                    const float *c = v->rgba + 4 * o;
                    double at = corrected_alpha(c[3], h / ((b - f) / list_cos(v, &cO, lx, ly)));
                    for (int m = 0; m < 3; ++m) C[m] += T * at * c[m];
                    T *= 1.0 - at;
                    break;
                }
            }
        }
        o4[0] = C[0]; o4[1] = C[1]; o4[2] = C[2]; o4[3] = 1.0 - T;
    }
    return 0;
}

int or_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
