/*
 * FP64 CPU oracle for the hybrid VPL method of "A Virtual Point Light
 * Generation Method in Close-Range Area" (Jin, Wang, Zheng, Hua, Huo).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing on the product path may call, link or
 * load this file: it is used by the tests, by the smoke check and by the
 * CPU-baseline leg of the benchmark.  It shares no code, header, table or
 * helper with the GPU library; both read the same float32 input arrays.
 *
 * Plain and slow on purpose: every quantity is computed in double precision
 * straight from its definition, with no blocking, fusion or reordering.
 *
 *   visibility   V(x,y) of eq. (1) and eq. (2): brute force over every
 *                triangle, or over this file's own median-split BVH (checked
 *                against brute force by the tests)
 *   G-buffer     closest hit of one primary ray per pixel centre
 *   gather       eq. (1) without the direct term: per pixel, the sum over all
 *                VPLs of (albedo/pi) * I_k * min(C, cos_p cos_k / r^2) * V
 *   direct       the direct term L_e(y) of eq. (1) with the light model of
 *                eq. (2)
 *   generation   Section "Close-Range VPL Sampling": near/far split of the
 *                one-sided faces, Morton-sorted area CDF cut into K strata,
 *                eq. (2) for the patch VPLs, and a sparse quasi-random walk
 *                (instant radiosity) that keeps far hits only.
 *
 * Build with -ffp-contract=off: every integer decision (near/far, patch,
 * stratum, Halton index, hit triangle) is taken in FP64 with the operation
 * order written here, and the GPU path takes the same decisions in the same
 * order.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define OR_PI 3.14159265358979323846
#define OR_MAX_STACK 256

typedef struct { double x, y, z; } v3;

static v3 mk(double x, double y, double z) { v3 r; r.x = x; r.y = y; r.z = z; return r; }
static v3 vadd(v3 a, v3 b) { return mk(a.x + b.x, a.y + b.y, a.z + b.z); }
static v3 vsub(v3 a, v3 b) { return mk(a.x - b.x, a.y - b.y, a.z - b.z); }
static v3 vscl(v3 a, double s) { return mk(a.x * s, a.y * s, a.z * s); }
static double vdot(v3 a, v3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
static v3 vcross(v3 a, v3 b)
{
    return mk(a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x);
}
static v3 vnorm(v3 a)
{
    double l = sqrt(vdot(a, a));
    return mk(a.x / l, a.y / l, a.z / l);
}
static v3 vld(const float* p) { return mk((double)p[0], (double)p[1], (double)p[2]); }
static v3 vldd(const double* p) { return mk(p[0], p[1], p[2]); }
static double dmin(double a, double b) { return a < b ? a : b; }
static double dmax(double a, double b) { return a > b ? a : b; }

/* ------------------------------------------------------------------------ */
/* scene                                                                    */
/* ------------------------------------------------------------------------ */

typedef struct {
    v3 lo, hi;
    int left, right; /* children (inner) */
    int first, count; /* triangle range in order[] (leaf iff count > 0) */
} onode;

typedef struct {
    int T;
    v3 *A, *B, *C, *e1, *e2, *n;
    double* rho;
    uint8_t* flags;
    v3 lo, hi;
    double diag;
    onode* nodes;
    int n_nodes;
    int* order;
    int use_bvh;
} oscene;

static const double* g_sort_key;
static int cmp_key(const void* a, const void* b)
{
    int ia = *(const int*)a, ib = *(const int*)b;
    double ka = g_sort_key[ia], kb = g_sort_key[ib];
    if (ka < kb) return -1;
    if (ka > kb) return 1;
    return (ia > ib) - (ia < ib);
}

/* Median-split BVH: split the longest centroid axis at the median, leaves of
 * at most 4 triangles, boxes padded outward so FP64 slab tests never drop a
 * triangle that the exact box contains. */
static int bvh_build(oscene* s, int first, int count, double* cen, double* key, double pad)
{
    int id = s->n_nodes++;
    onode* nd = &s->nodes[id];
    v3 lo = mk(INFINITY, INFINITY, INFINITY), hi = mk(-INFINITY, -INFINITY, -INFINITY);
    v3 clo = lo, chi = hi;
    for (int i = first; i < first + count; i++) {
        int t = s->order[i];
        v3 p[3] = {s->A[t], s->B[t], s->C[t]};
        for (int k = 0; k < 3; k++) {
            lo = mk(dmin(lo.x, p[k].x), dmin(lo.y, p[k].y), dmin(lo.z, p[k].z));
            hi = mk(dmax(hi.x, p[k].x), dmax(hi.y, p[k].y), dmax(hi.z, p[k].z));
        }
        v3 c = vldd(&cen[3 * t]);
        clo = mk(dmin(clo.x, c.x), dmin(clo.y, c.y), dmin(clo.z, c.z));
        chi = mk(dmax(chi.x, c.x), dmax(chi.y, c.y), dmax(chi.z, c.z));
    }
    nd->lo = mk(lo.x - pad, lo.y - pad, lo.z - pad);
    nd->hi = mk(hi.x + pad, hi.y + pad, hi.z + pad);
    if (count <= 4) {
        nd->first = first;
        nd->count = count;
        nd->left = nd->right = -1;
        return id;
    }
    v3 ext = vsub(chi, clo);
    int axis = 0;
    if (ext.y > ext.x) axis = 1;
    if (ext.z > (axis == 0 ? ext.x : ext.y)) axis = 2;
    for (int i = first; i < first + count; i++) {
        int t = s->order[i];
        key[t] = cen[3 * t + axis];
    }
    g_sort_key = key;
    qsort(s->order + first, (size_t)count, sizeof(int), cmp_key);
    int half = count / 2;
    nd->first = 0;
    nd->count = 0;
    int l = bvh_build(s, first, half, cen, key, pad);
    int r = bvh_build(s, first + half, count - half, cen, key, pad);
    s->nodes[id].left = l;
    s->nodes[id].right = r;
    return id;
}

void* oracle_scene_create(const float* tri, const float* albedo, const uint8_t* flags, int T, int use_bvh)
{
    oscene* s = (oscene*)calloc(1, sizeof(oscene));
    s->T = T;
    s->A = (v3*)malloc(sizeof(v3) * (size_t)(T > 0 ? T : 1));
    s->B = (v3*)malloc(sizeof(v3) * (size_t)(T > 0 ? T : 1));
    s->C = (v3*)malloc(sizeof(v3) * (size_t)(T > 0 ? T : 1));
    s->e1 = (v3*)malloc(sizeof(v3) * (size_t)(T > 0 ? T : 1));
    s->e2 = (v3*)malloc(sizeof(v3) * (size_t)(T > 0 ? T : 1));
    s->n = (v3*)malloc(sizeof(v3) * (size_t)(T > 0 ? T : 1));
    s->rho = (double*)malloc(sizeof(double) * 3 * (size_t)(T > 0 ? T : 1));
    s->flags = (uint8_t*)malloc((size_t)(T > 0 ? T : 1));
    s->lo = mk(INFINITY, INFINITY, INFINITY);
    s->hi = mk(-INFINITY, -INFINITY, -INFINITY);
    for (int t = 0; t < T; t++) {
        s->A[t] = vld(tri + 9 * t);
        s->B[t] = vld(tri + 9 * t + 3);
        s->C[t] = vld(tri + 9 * t + 6);
        s->e1[t] = vsub(s->B[t], s->A[t]);
        s->e2[t] = vsub(s->C[t], s->A[t]);
        /* one-sided face: counter-clockwise winding is the front */
        s->n[t] = vnorm(vcross(s->e1[t], s->e2[t]));
        for (int k = 0; k < 3; k++) s->rho[3 * t + k] = (double)albedo[3 * t + k];
        s->flags[t] = flags[t];
        v3 p[3] = {s->A[t], s->B[t], s->C[t]};
        for (int k = 0; k < 3; k++) {
            s->lo = mk(dmin(s->lo.x, p[k].x), dmin(s->lo.y, p[k].y), dmin(s->lo.z, p[k].z));
            s->hi = mk(dmax(s->hi.x, p[k].x), dmax(s->hi.y, p[k].y), dmax(s->hi.z, p[k].z));
        }
    }
    v3 ext = vsub(s->hi, s->lo);
    s->diag = T > 0 ? sqrt(vdot(ext, ext)) : 0.0;
    s->use_bvh = use_bvh && T > 0;
    if (s->use_bvh) {
        double* cen = (double*)malloc(sizeof(double) * 3 * (size_t)T);
        double* key = (double*)malloc(sizeof(double) * (size_t)T);
        for (int t = 0; t < T; t++) {
            cen[3 * t + 0] = (s->A[t].x + s->B[t].x + s->C[t].x) / 3.0;
            cen[3 * t + 1] = (s->A[t].y + s->B[t].y + s->C[t].y) / 3.0;
            cen[3 * t + 2] = (s->A[t].z + s->B[t].z + s->C[t].z) / 3.0;
        }
        s->order = (int*)malloc(sizeof(int) * (size_t)T);
        for (int t = 0; t < T; t++) s->order[t] = t;
        s->nodes = (onode*)malloc(sizeof(onode) * (size_t)(2 * T));
        s->n_nodes = 0;
        bvh_build(s, 0, T, cen, key, 1e-7 * s->diag + 1e-300);
        free(cen);
        free(key);
    }
    return s;
}

void oracle_scene_destroy(void* h)
{
    oscene* s = (oscene*)h;
    if (!s) return;
    free(s->A); free(s->B); free(s->C); free(s->e1); free(s->e2); free(s->n);
    free(s->rho); free(s->flags); free(s->nodes); free(s->order);
    free(s);
}

int oracle_scene_bvh_nodes(void* h) { return ((oscene*)h)->n_nodes; }

void oracle_face_normals(void* h, double* out)
{
    oscene* s = (oscene*)h;
    for (int t = 0; t < s->T; t++) {
        out[3 * t] = s->n[t].x;
        out[3 * t + 1] = s->n[t].y;
        out[3 * t + 2] = s->n[t].z;
    }
}

/* ------------------------------------------------------------------------ */
/* ray / triangle and ray / box                                             */
/* ------------------------------------------------------------------------ */

/* Moller-Trumbore in FP64 with a fixed operation order.  The hit is the
 * closed triangle u >= 0, v >= 0, u + v <= 1; a ray parallel to the plane
 * (det == 0) never hits.  Returns the ray parameter through *t. */
static int tri_isect(const oscene* s, int t, v3 o, v3 d, double* tt, double* uu, double* vv)
{
    v3 e1 = s->e1[t], e2 = s->e2[t];
    v3 pvec = vcross(d, e2);
    double det = vdot(e1, pvec);
    if (det == 0.0) return 0;
    double inv = 1.0 / det;
    v3 tvec = vsub(o, s->A[t]);
    double u = vdot(tvec, pvec) * inv;
    if (u < 0.0 || u > 1.0) return 0;
    v3 qvec = vcross(tvec, e1);
    double v = vdot(d, qvec) * inv;
    if (v < 0.0 || u + v > 1.0) return 0;
    *tt = vdot(e2, qvec) * inv;
    *uu = u;
    *vv = v;
    return 1;
}

static int box_isect(const onode* nd, v3 o, v3 d, double tmin, double tmax)
{
    double oo[3] = {o.x, o.y, o.z}, dd[3] = {d.x, d.y, d.z};
    double lo[3] = {nd->lo.x, nd->lo.y, nd->lo.z}, hi[3] = {nd->hi.x, nd->hi.y, nd->hi.z};
    for (int k = 0; k < 3; k++) {
        if (dd[k] == 0.0) {
            if (oo[k] < lo[k] || oo[k] > hi[k]) return 0;
            continue;
        }
        double t0 = (lo[k] - oo[k]) / dd[k], t1 = (hi[k] - oo[k]) / dd[k];
        if (t0 > t1) { double tmp = t0; t0 = t1; t1 = tmp; }
        tmin = dmax(tmin, t0);
        tmax = dmin(tmax, t1);
        if (tmin > tmax) return 0;
    }
    return 1;
}

/* Visibility of eq. (1)/(2): the segment x + s (y - x), s in (eps, 1 - eps),
 * is blocked iff some triangle other than the two host triangles crosses it.
 * Occlusion is two-sided and emitters occlude. Returns 1 if visible. */
static int visible(const oscene* s, v3 x, int tx, v3 y, int ty, double eps)
{
    v3 d = vsub(y, x);
    double lo = eps, hi = 1.0 - eps;
    if (!s->use_bvh) {
        for (int t = 0; t < s->T; t++) {
            double tt, u, v;
            if (t == tx || t == ty) continue;
            if (tri_isect(s, t, x, d, &tt, &u, &v) && tt > lo && tt < hi) return 0;
        }
        return 1;
    }
    int stack[OR_MAX_STACK];
    int sp = 0;
    stack[sp++] = 0;
    while (sp > 0) {
        const onode* nd = &s->nodes[stack[--sp]];
        if (!box_isect(nd, x, d, lo, hi)) continue;
        if (nd->count > 0) {
            for (int i = nd->first; i < nd->first + nd->count; i++) {
                int t = s->order[i];
                double tt, u, v;
                if (t == tx || t == ty) continue;
                if (tri_isect(s, t, x, d, &tt, &u, &v) && tt > lo && tt < hi) return 0;
            }
        } else {
            stack[sp++] = nd->left;
            stack[sp++] = nd->right;
        }
    }
    return 1;
}

/* Closest hit with t in (tmin, tmax); ties go to the smaller triangle index.
 * Triangle `ex` is skipped, and so are all emitters when skip_emit is set. */
static int closest(const oscene* s, v3 o, v3 d, double tmin, double tmax, int ex, int skip_emit,
                   double* tb, double* ub, double* vb)
{
    int best = -1;
    double bt = tmax, bu = 0, bv = 0;
    if (!s->use_bvh) {
        for (int t = 0; t < s->T; t++) {
            double tt, u, v;
            if (t == ex || (skip_emit && (s->flags[t] & 1))) continue;
            if (tri_isect(s, t, o, d, &tt, &u, &v) && tt > tmin && tt < tmax) {
                if (best < 0 || tt < bt || (tt == bt && t < best)) { best = t; bt = tt; bu = u; bv = v; }
            }
        }
    } else {
        int stack[OR_MAX_STACK];
        int sp = 0;
        stack[sp++] = 0;
        while (sp > 0) {
            const onode* nd = &s->nodes[stack[--sp]];
            if (!box_isect(nd, o, d, tmin, best >= 0 ? bt : tmax)) continue;
            if (nd->count > 0) {
                for (int i = nd->first; i < nd->first + nd->count; i++) {
                    int t = s->order[i];
                    double tt, u, v;
                    if (t == ex || (skip_emit && (s->flags[t] & 1))) continue;
                    if (tri_isect(s, t, o, d, &tt, &u, &v) && tt > tmin && tt < tmax) {
                        if (best < 0 || tt < bt || (tt == bt && t < best)) { best = t; bt = tt; bu = u; bv = v; }
                    }
                }
            } else {
                stack[sp++] = nd->left;
                stack[sp++] = nd->right;
            }
        }
    }
    *tb = bt; *ub = bu; *vb = bv;
    return best;
}

/* ------------------------------------------------------------------------ */
/* visibility queries                                                       */
/* ------------------------------------------------------------------------ */

/* vis[i] = V(x_i, y_i) for n segments (x, y as float32 xyz triples). */
void oracle_visibility(void* h, const float* x, const int32_t* tx, const float* y, const int32_t* ty,
                       int64_t n, double eps, uint8_t* vis)
{
    const oscene* s = (const oscene*)h;
#pragma omp parallel for schedule(dynamic, 256)
    for (int64_t i = 0; i < n; i++)
        vis[i] = (uint8_t)visible(s, vld(x + 3 * i), tx[i], vld(y + 3 * i), ty[i], eps);
}

/* A pair is grazing when moving one endpoint by delta along a coordinate
 * axis (12 variants) changes its visibility. */
void oracle_grazing(void* h, const float* x, const int32_t* tx, const float* y, const int32_t* ty,
                    int64_t n, double eps, double delta, uint8_t* out)
{
    const oscene* s = (const oscene*)h;
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t i = 0; i < n; i++) {
        v3 xp = vld(x + 3 * i), yp = vld(y + 3 * i);
        int v0 = visible(s, xp, tx[i], yp, ty[i], eps);
        int g = 0;
        for (int k = 0; k < 12 && !g; k++) {
            v3 off = mk(0, 0, 0);
            double sg = (k & 1) ? -delta : delta;
            int ax = (k >> 1) % 3;
            if (ax == 0) off.x = sg; else if (ax == 1) off.y = sg; else off.z = sg;
            v3 xa = xp, ya = yp;
            if (k < 6) xa = vadd(xa, off); else ya = vadd(ya, off);
            if (visible(s, xa, tx[i], ya, ty[i], eps) != v0) g = 1;
        }
        out[i] = (uint8_t)g;
    }
}

/* ------------------------------------------------------------------------ */
/* camera                                                                   */
/* ------------------------------------------------------------------------ */

typedef struct { v3 eye, f, r, u; double th, tx; int W, H; } ocam;

/* cam = eye[3], target[3], up[3], vfov_deg, width, height.  Basis
 * f = normalize(target - eye), r = normalize(f x up), u = r x f;
 * th = tan(vfov/2), tx = th * W/H. */
static ocam make_cam(const double* c)
{
    ocam k;
    k.eye = vldd(c);
    k.f = vnorm(vsub(vldd(c + 3), k.eye));
    k.r = vnorm(vcross(k.f, vldd(c + 6)));
    k.u = vcross(k.r, k.f);
    k.W = (int)c[10];
    k.H = (int)c[11];
    k.th = tan(c[9] * (OR_PI / 360.0));
    k.tx = k.th * ((double)k.W / (double)k.H);
    return k;
}

static v3 pixel_dir(const ocam* k, int i, int j)
{
    double sx = (2.0 * ((double)i + 0.5) / (double)k->W - 1.0) * k->tx;
    double sy = (1.0 - 2.0 * ((double)j + 0.5) / (double)k->H) * k->th;
    return vadd(vadd(k->f, vscl(k->r, sx)), vscl(k->u, sy));
}

/* G-buffer: closest hit (t > 0) of the ray through each pixel centre; the
 * position is the barycentric point on the hit triangle, the normal the
 * unflipped face normal.  tri = -1 and zeros on a miss. */
void oracle_gbuffer(void* h, const double* cam, double* pos, double* nrm, double* alb, int32_t* tri)
{
    const oscene* s = (const oscene*)h;
    ocam k = make_cam(cam);
    int64_t P = (int64_t)k.W * k.H;
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t p = 0; p < P; p++) {
        int i = (int)(p % k.W), j = (int)(p / k.W);
        v3 d = pixel_dir(&k, i, j);
        double tb, u, v;
        int t = closest(s, k.eye, d, 0.0, INFINITY, -1, 0, &tb, &u, &v);
        tri[p] = t;
        if (t < 0) {
            for (int c = 0; c < 3; c++) pos[3 * p + c] = nrm[3 * p + c] = alb[3 * p + c] = 0.0;
            continue;
        }
        v3 x = vadd(vadd(s->A[t], vscl(s->e1[t], u)), vscl(s->e2[t], v));
        pos[3 * p] = x.x; pos[3 * p + 1] = x.y; pos[3 * p + 2] = x.z;
        nrm[3 * p] = s->n[t].x; nrm[3 * p + 1] = s->n[t].y; nrm[3 * p + 2] = s->n[t].z;
        for (int c = 0; c < 3; c++) alb[3 * p + c] = s->rho[3 * t + c];
    }
}

/* Pixels whose hit triangle changes when the ray direction is tilted by
 * `delta` (relative) along the camera's right or up axis: silhouettes and
 * triangle edges where FP32 and FP64 may legitimately pick different faces. */
void oracle_gbuffer_edges(void* h, const double* cam, double delta, uint8_t* out)
{
    const oscene* s = (const oscene*)h;
    ocam k = make_cam(cam);
    int64_t P = (int64_t)k.W * k.H;
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t p = 0; p < P; p++) {
        int i = (int)(p % k.W), j = (int)(p / k.W);
        v3 d = pixel_dir(&k, i, j);
        double l = sqrt(vdot(d, d)), tb, u, v;
        int t0 = closest(s, k.eye, d, 0.0, INFINITY, -1, 0, &tb, &u, &v);
        int e = 0;
        for (int q = 0; q < 4 && !e; q++) {
            v3 ax = (q < 2) ? k.r : k.u;
            v3 dq = vadd(d, vscl(ax, (q & 1 ? -delta : delta) * l));
            if (closest(s, k.eye, dq, 0.0, INFINITY, -1, 0, &tb, &u, &v) != t0) e = 1;
        }
        out[p] = (uint8_t)e;
    }
}

/* ------------------------------------------------------------------------ */
/* gather: eq. (1), indirect part                                           */
/* ------------------------------------------------------------------------ */

/* For each of n_px G-buffer entries (position, normal, albedo, tri as float32
 * / int32 AoS), L = (albedo / pi) * sum_k I_k * min(C, max(0, n_p.d) *
 * max(0, -n_k.d) / |d|^4) * V(x_p, y_k), d = y_k - x_p, summed over k in
 * order.  Invalid pixels (tri < 0) give 0.  Optional overrides (sorted by
 * pixel, then VPL) replace V for listed pairs.  nthreads <= 0: OpenMP default. */
void oracle_gather(void* h, const float* gpos, const float* gnrm, const float* galb, const int32_t* gtri,
                   int64_t n_px, const float* vpos, const float* vnrm, const float* vI, const int32_t* vtri,
                   int M, double C, double eps, const int32_t* ov_px, const int32_t* ov_vpl,
                   const uint8_t* ov_vis, int64_t n_ov, int nthreads, double* L)
{
    const oscene* s = (const oscene*)h;
#ifdef _OPENMP
    int nt = nthreads > 0 ? nthreads : omp_get_max_threads();
#pragma omp parallel for schedule(dynamic, 1) num_threads(nt)
#endif
    for (int64_t p = 0; p < n_px; p++) {
        double acc[3] = {0, 0, 0};
        int tp = gtri[p];
        if (tp >= 0) {
            v3 x = vld(gpos + 3 * p), np = vld(gnrm + 3 * p);
            /* overrides of this pixel */
            int64_t lo = 0, hi = n_ov;
            while (lo < hi) { int64_t mid = (lo + hi) / 2; if (ov_px[mid] < p) lo = mid + 1; else hi = mid; }
            int64_t oi = lo;
            for (int k = 0; k < M; k++) {
                v3 y = vld(vpos + 3 * k), nk = vld(vnrm + 3 * k);
                v3 d = vsub(y, x);
                double r2 = vdot(d, d);
                double cp = vdot(np, d);
                double ck = -vdot(nk, d);
                while (oi < n_ov && ov_px[oi] == p && ov_vpl[oi] < k) oi++;
                if (!(cp > 0.0 && ck > 0.0)) continue;
                double g = dmin(C, (cp * ck) / (r2 * r2));
                int vis;
                if (oi < n_ov && ov_px[oi] == p && ov_vpl[oi] == k) vis = ov_vis[oi];
                else vis = visible(s, x, tp, y, vtri[k], eps);
                if (!vis) continue;
                for (int c = 0; c < 3; c++) acc[c] += (double)vI[3 * k + c] * g;
            }
            for (int c = 0; c < 3; c++) acc[c] = ((double)galb[3 * p + c] / OR_PI) * acc[c];
        }
        for (int c = 0; c < 3; c++) L[3 * p + c] = acc[c];
    }
}

/* Visibility of every (pixel, VPL) pair, computed for all pairs (no
 * geometry-term culling).  vis is n_px x M, row-major. */
void oracle_vis_matrix(void* h, const float* gpos, const int32_t* gtri, int64_t n_px, const float* vpos,
                       const int32_t* vtri, int M, double eps, uint8_t* vis)
{
    const oscene* s = (const oscene*)h;
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t p = 0; p < n_px; p++) {
        v3 x = vld(gpos + 3 * p);
        for (int k = 0; k < M; k++)
            vis[p * M + k] = gtri[p] < 0 ? 0 : (uint8_t)visible(s, x, gtri[p], vld(vpos + 3 * k), vtri[k], eps);
    }
}

/* ------------------------------------------------------------------------ */
/* generation: Section "Close-Range VPL Sampling"                           */
/* ------------------------------------------------------------------------ */

/* Radical inverse of i in base b, as an exact integer ratio num / b^m. */
double oracle_halton(int b, int64_t i)
{
    uint64_t num = 0, den = 1, q = (uint64_t)i;
    while (q > 0) {
        num = num * (uint64_t)b + q % (uint64_t)b;
        den *= (uint64_t)b;
        q /= (uint64_t)b;
    }
    return (double)num / (double)den;
}

/* Refinement level of a triangle: the smallest n >= 1 with (n h)^2 >= the
 * longest squared edge, so every patch edge is at most h. */
static int patch_level(const oscene* s, int t, double h)
{
    v3 a = vsub(s->B[t], s->A[t]), b = vsub(s->C[t], s->B[t]), c = vsub(s->A[t], s->C[t]);
    double m2 = dmax(dmax(vdot(a, a), vdot(b, b)), vdot(c, c));
    int n = (int)floor(sqrt(m2) / h) - 1;
    if (n < 1) n = 1;
    while (((double)n * h) * ((double)n * h) < m2) n++;
    return n;
}

int64_t oracle_patch_count(void* h, double patch_h)
{
    const oscene* s = (const oscene*)h;
    int64_t total = 0;
    for (int t = 0; t < s->T; t++) {
        int64_t n = patch_level(s, t, patch_h);
        total += n * n;
    }
    return total;
}

/* grid point A + (B - A) a/n + (C - A) b/n */
static v3 grid_pt(const oscene* s, int t, int n, int a, int b)
{
    return vadd(vadd(s->A[t], vscl(s->e1[t], (double)a / (double)n)), vscl(s->e2[t], (double)b / (double)n));
}

/* Patch (a, b, down) of triangle t: up = (a,b),(a+1,b),(a,b+1); down =
 * (a+1,b),(a+1,b+1),(a,b+1).  Within a triangle patches are numbered by row
 * b, then a, up before down: local index b (2n - b) + 2a + down. */
static void patch_verts(const oscene* s, int t, int n, int a, int b, int down, v3* P)
{
    if (!down) {
        P[0] = grid_pt(s, t, n, a, b); P[1] = grid_pt(s, t, n, a + 1, b); P[2] = grid_pt(s, t, n, a, b + 1);
    } else {
        P[0] = grid_pt(s, t, n, a + 1, b); P[1] = grid_pt(s, t, n, a + 1, b + 1); P[2] = grid_pt(s, t, n, a, b + 1);
    }
}

static void local_to_ab(int n, int local, int* a, int* b, int* down)
{
    int r = 0;
    while ((int64_t)(r + 1) * (2 * n - (r + 1)) <= local) r++;
    int rem = local - r * (2 * n - r);
    *b = r;
    *a = rem / 2;
    *down = rem & 1;
}

/* Near region (Section "Close-Range VPL Sampling"): the patch centroid lies
 * in front of the camera, inside the view frustum, and closer than d_near. */
static int is_near(const ocam* k, v3 c, double dn)
{
    v3 v = vsub(c, k->eye);
    double z = vdot(v, k->f);
    if (!(z > 0.0)) return 0;
    if (!(fabs(vdot(v, k->r)) <= z * k->tx)) return 0;
    if (!(fabs(vdot(v, k->u)) <= z * k->th)) return 0;
    return vdot(v, v) < dn * dn;
}

typedef struct {
    int kind;
    v3 pos, eu, ev, nl, lc;
    double power[3];
} olight;

/* light = kind, pos[3], edge_u[3], edge_v[3], power[3] */
static olight make_light(const double* l)
{
    olight L;
    L.kind = (int)l[0];
    L.pos = vldd(l + 1);
    L.eu = vldd(l + 4);
    L.ev = vldd(l + 7);
    for (int c = 0; c < 3; c++) L.power[c] = l[10 + c];
    if (L.kind == 1) {
        L.nl = vnorm(vcross(L.eu, L.ev));
        L.lc = vadd(vadd(L.pos, vscl(L.eu, 0.5)), vscl(L.ev, 0.5));
    } else {
        L.nl = mk(0, 0, 0);
        L.lc = L.pos;
    }
    return L;
}

/* ------------------------------------------------------------------------ */
/* direct term L_e(y) of eq. (1)                                            */
/* ------------------------------------------------------------------------ */

/* Sample points of the light, as eq. (2) uses them: the point light itself,
 * or the 16 cell centres pos + eu (i + 1/2)/4 + ev (j + 1/2)/4 (cell j*4+i)
 * of the quad.  Returns the count (1 or 16); xyz gets 3 doubles each. */
int oracle_light_samples(const double* light, double* xyz)
{
    olight L = make_light(light);
    if (L.kind == 0) {
        xyz[0] = L.pos.x; xyz[1] = L.pos.y; xyz[2] = L.pos.z;
        return 1;
    }
    for (int j = 0; j < 16; j++) {
        v3 lj = vadd(vadd(L.pos, vscl(L.eu, ((double)(j % 4) + 0.5) / 4.0)), vscl(L.ev, ((double)(j / 4) + 0.5) / 4.0));
        xyz[3 * j] = lj.x; xyz[3 * j + 1] = lj.y; xyz[3 * j + 2] = lj.z;
    }
    return 16;
}

/* Direct illumination L_e(y) of eq. (1) at each of n_px G-buffer entries:
 * (albedo / pi) * Phi * g(x, n) with the light model of eq. (2): for the
 * point light g = max(0, n.w) / (4 pi r^3), w = pos - x; for the quad,
 * g = (1/16) sum_j max(0, n.w_j) max(0, -n_l.w_j) / (pi r_j^4) over the cell
 * centres y_j, w_j = y_j - x.  Each sample counts only if V(x, y_j) = 1
 * (host triangle excluded, the light's own triangles not).  Optional
 * overrides (sorted by pixel, then sample) replace V for listed pairs. */
void oracle_direct(void* h, const float* gpos, const float* gnrm, const float* galb, const int32_t* gtri,
                   int64_t n_px, const double* light, double eps, const int32_t* ov_px, const int32_t* ov_s,
                   const uint8_t* ov_vis, int64_t n_ov, double* Lout)
{
    const oscene* s = (const oscene*)h;
    olight L = make_light(light);
    double ys[48];
    int ns = oracle_light_samples(light, ys);
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t p = 0; p < n_px; p++) {
        double g = 0.0;
        int tp = gtri[p];
        if (tp >= 0) {
            v3 x = vld(gpos + 3 * p), np = vld(gnrm + 3 * p);
            int64_t lo = 0, hi = n_ov;
            while (lo < hi) { int64_t mid = (lo + hi) / 2; if (ov_px[mid] < p) lo = mid + 1; else hi = mid; }
            int64_t oi = lo;
            for (int j = 0; j < ns; j++) {
                v3 y = vldd(ys + 3 * j);
                v3 w = vsub(y, x);
                double r2 = vdot(w, w);
                double cx = vdot(np, w);
                double cl = L.kind == 0 ? 1.0 : -vdot(L.nl, w);
                while (oi < n_ov && ov_px[oi] == p && ov_s[oi] < j) oi++;
                if (!(cx > 0.0 && cl > 0.0)) continue;
                int vis;
                if (oi < n_ov && ov_px[oi] == p && ov_s[oi] == j) vis = ov_vis[oi];
                else vis = visible(s, x, tp, y, -1, eps);
                if (!vis) continue;
                if (L.kind == 0) g += cx / ((4.0 * OR_PI) * (r2 * sqrt(r2)));
                else g += (cx * cl) / (OR_PI * (r2 * r2));
            }
            if (L.kind == 1) g = g / 16.0;
        }
        for (int c = 0; c < 3; c++)
            Lout[3 * p + c] = tp >= 0 ? ((double)galb[3 * p + c] / OR_PI) * (L.power[c] * g) : 0.0;
    }
}

static uint32_t morton30(int cx, int cy, int cz)
{
    uint32_t key = 0;
    for (int b = 0; b < 10; b++) {
        key |= (uint32_t)((cx >> b) & 1) << (3 * b);
        key |= (uint32_t)((cy >> b) & 1) << (3 * b + 1);
        key |= (uint32_t)((cz >> b) & 1) << (3 * b + 2);
    }
    return key;
}

static int cell_of(double c, double lo, double h)
{
    double f = floor((c - lo) / h);
    if (f < 0.0) f = 0.0;
    if (f > 1023.0) f = 1023.0;
    return (int)f;
}

typedef struct { uint32_t key; int32_t idx; } kpair;
static int cmp_kpair(const void* a, const void* b)
{
    const kpair* x = (const kpair*)a;
    const kpair* y = (const kpair*)b;
    if (x->key != y->key) return x->key < y->key ? -1 : 1;
    return (x->idx > y->idx) - (x->idx < y->idx);
}

/* Duff et al. 2017 orthonormal basis around n; returns x b1 + y b2 + z n. */
static v3 onb_dir(v3 n, double x, double y, double z)
{
    double sign = copysign(1.0, n.z);
    double a = -1.0 / (sign + n.z);
    double b = n.x * n.y * a;
    v3 b1 = mk(1.0 + sign * n.x * n.x * a, sign * b, -sign * n.x);
    v3 b2 = mk(b, sign + n.y * n.y * a, -n.y);
    return mk(x * b1.x + y * b2.x + z * n.x, x * b1.y + y * b2.y + z * n.y, x * b1.z + y * b2.z + z * n.z);
}

/* cosine-weighted direction about n (Malley: uniform disk lifted to the hemisphere) */
static v3 cos_dir(v3 n, double u1, double u2)
{
    double r = sqrt(u1);
    double ph = (2.0 * OR_PI) * u2;
    return onb_dir(n, r * cos(ph), r * sin(ph), sqrt(dmax(0.0, 1.0 - u1)));
}

static const int PRIMES[8] = {2, 3, 5, 7, 11, 13, 17, 19};

/* stats layout */
enum {
    ST_PATCHES = 0, ST_NEAR, ST_ELIGIBLE, ST_Q, ST_KEFF, ST_NFAR_TARGET, ST_NFAR, ST_NPATHS,
    ST_B1, ST_B2, ST_B3, ST_FLAGS, ST_NEAR_DISCARDED, ST_COUNT
};

/* Mean albedo of the scene for Keller's path schedule: the face-area-weighted
 * mean, over the faces that do not emit, of the mean of the three channels
 * (0 when those faces have no area). */
double oracle_rho_bar(void* h)
{
    const oscene* s = (const oscene*)h;
    double num = 0.0, den = 0.0;
    for (int t = 0; t < s->T; t++) {
        if (s->flags[t] & 1) continue;
        v3 cr = vcross(s->e1[t], s->e2[t]);
        double a = 0.5 * sqrt(vdot(cr, cr));
        num += a * (((s->rho[3 * t] + s->rho[3 * t + 1]) + s->rho[3 * t + 2]) / 3.0);
        den += a;
    }
    return den > 0.0 ? num / den : 0.0;
}

/* Eq. (2)'s light factor at point y (normal nk, on triangle t): Phi-free
 * irradiance per unit power, V cos / (4 pi r^2) for the point light, or the
 * mean over the 16 quad cells of V cos_l cos / (pi r^2). */
static double light_factor(const oscene* s, const olight* L, v3 y, v3 nk, int t, double eps)
{
    double gsum = 0.0;
    if (L->kind == 0) {
        v3 w = vsub(L->pos, y);
        double r2w = vdot(w, w);
        double r = sqrt(r2w);
        double ck = vdot(nk, w) / r;
        if (ck > 0.0 && visible(s, y, t, L->pos, -1, eps)) gsum = ck / ((4.0 * OR_PI) * r2w);
    } else {
        for (int j = 0; j < 16; j++) {
            v3 lj = vadd(vadd(L->pos, vscl(L->eu, ((double)(j % 4) + 0.5) / 4.0)),
                         vscl(L->ev, ((double)(j / 4) + 0.5) / 4.0));
            v3 w = vsub(lj, y);
            double r2w = vdot(w, w);
            double r = sqrt(r2w);
            double cl = -vdot(L->nl, w) / r;
            double ck = vdot(nk, w) / r;
            if (cl > 0.0 && ck > 0.0 && visible(s, y, t, lj, -1, eps)) gsum += (cl * ck) / (OR_PI * r2w);
        }
        gsum = gsum / 16.0;
    }
    return gsum;
}

/*
 * Full VPL generation.  cam = eye, target, up, vfov_deg, W, H; light = kind,
 * pos, edge_u, edge_v, power; ip = k_near, n_far, max_bounces, max_paths, walk_near,
 * jitter, brightness, walk_schedule; dp = d_near, patch_h.
 *
 * Readings of the paper's generation steps (Section "Realization of VPL
 * Generation Algorithm Based on Patch" and the flow steps (1)-(3)):
 *   walk_near  0: every walk hit on a near patch is discarded and the path
 *                 continues (flow step (3) as written);
 *              1: only first-bounce near hits are discarded (later ones are
 *                 kept as walk VPLs);
 *              2: a near hit is discarded and ends its path.
 *   jitter     0: stratum k's target is its midpoint floor((2k+1) f(N) / 2K);
 *              1: the target is B_k + floor(xi_k (B_{k+1} - B_k)) with the
 *                 stratum bounds B_k = floor(k f(N) / K) and xi_k the Halton
 *                 base-5 value of k + 1.
 *   walk_schedule 0: paths run until n_far far VPLs exist (the last path
 *                 cut there), fluxes divided by the number of paths;
 *              1: Keller's schedule for instant radiosity: N = floor(n_far /
 *                 sum_{j < max_bounces} rb^j) paths with rb the scene's mean
 *                 albedo (area-weighted over the faces that do not emit, mean
 *                 of the three channels); path i goes on to bounce b only if
 *                 i <= floor(rb^(b-1) N), and a deposit at bounce b carries
 *                 Phi prod(rho) / (N rb^(b-1)) (the paths that stop stand for
 *                 the light the others carry on).
 *   brightness 0: the VPL's flux is eq. (2) at its own point with the area
 *                 D = f(N) / K it stands for;
 *              1: the flux is eq. (2) summed over the set of patches of its
 *                 stratum, each patch evaluated at its centroid with the part
 *                 of its area that lies in [B_k, B_{k+1}) (a patch spanning
 *                 several strata shares its area among their VPLs).
 *
 * Outputs (caller-allocated):
 *   patch_off  int64 [T + 1]        first global patch index of each triangle
 *   pflags     uint8 [n_patches]    bit0 near, bit1 eligible
 *   sorted     int32 [n_patches]    eligible patches in (Morton key, index) order
 *   keys       uint32 [n_patches]   their Morton keys
 *   F          int64 [n_patches]    inclusive prefix of fixed-point areas
 *   m          int32 [k_near]       stratum -> position in `sorted`
 *   vpl_pos, vpl_nrm, vpl_I  double [cap*3];  vpl_tri int32 [cap]
 *   vpl_path int32 [cap] (0 for patch VPLs), vpl_bounce int32 [cap] (0 for patch VPLs)
 *   stats int64 [ST_COUNT]
 * Returns the number of VPLs written, or -1 if cap is too small.
 */
int oracle_generate(void* h, const double* cam, const double* light, const int64_t* ip, const double* dp,
                    double eps, int64_t* patch_off, uint8_t* pflags, int32_t* sorted, uint32_t* keys, int64_t* F,
                    int32_t* m, double* vpl_pos, double* vpl_nrm, double* vpl_I, int32_t* vpl_tri,
                    int32_t* vpl_path, int32_t* vpl_bounce, int64_t cap, int64_t* stats)
{
    const oscene* s = (const oscene*)h;
    ocam k = make_cam(cam);
    olight L = make_light(light);
    int K = (int)ip[0], n_far = (int)ip[1], maxb = (int)ip[2];
    int64_t max_paths = ip[3];
    int walk_near = (int)ip[4];
    int jitter = (int)ip[5], brightness = (int)ip[6], walk_schedule = (int)ip[7];
    double dn = dp[0], ph = dp[1];
    for (int i = 0; i < ST_COUNT; i++) stats[i] = 0;
    /* eight Halton bases: start (2 or 4 dimensions) + 2 per scatter */
    if (maxb < 1 || (L.kind == 0 ? 2 : 4) + 2 * (maxb - 1) > 8 || K < 0 || n_far < 0) return -2;
    if (walk_near < 0 || walk_near > 2 || jitter < 0 || jitter > 1 || brightness < 0 || brightness > 1 ||
        walk_schedule < 0 || walk_schedule > 1)
        return -2;

    /* step 1: refine every triangle into patches, classify near / eligible */
    int* level = (int*)malloc(sizeof(int) * (size_t)(s->T > 0 ? s->T : 1));
    patch_off[0] = 0;
    for (int t = 0; t < s->T; t++) {
        level[t] = patch_level(s, t, ph);
        patch_off[t + 1] = patch_off[t] + (int64_t)level[t] * level[t];
    }
    int64_t NP = patch_off[s->T];
    stats[ST_PATCHES] = NP;
    int64_t n_el = 0;
    kpair* kp = (kpair*)malloc(sizeof(kpair) * (size_t)(NP > 0 ? NP : 1));
    for (int t = 0; t < s->T; t++) {
        int n = level[t];
        for (int64_t loc = 0; loc < (int64_t)n * n; loc++) {
            int a, b, down;
            local_to_ab(n, (int)loc, &a, &b, &down);
            v3 P[3];
            patch_verts(s, t, n, a, b, down, P);
            v3 c = mk((P[0].x + P[1].x + P[2].x) / 3.0, (P[0].y + P[1].y + P[2].y) / 3.0,
                      (P[0].z + P[1].z + P[2].z) / 3.0);
            int64_t g = patch_off[t] + loc;
            uint8_t fl = 0;
            if (!(s->flags[t] & 1) && is_near(&k, c, dn)) {
                fl |= 1;
                int el = vdot(s->n[t], vsub(L.lc, c)) > 0.0;
                if (L.kind == 1) el = el && (vdot(L.nl, vsub(c, L.lc)) > 0.0);
                if (el) {
                    fl |= 2;
                    kp[n_el].key = morton30(cell_of(c.x, s->lo.x, ph), cell_of(c.y, s->lo.y, ph),
                                            cell_of(c.z, s->lo.z, ph));
                    kp[n_el].idx = (int32_t)g;
                    n_el++;
                }
            }
            pflags[g] = fl;
            if (fl & 1) stats[ST_NEAR]++;
        }
    }
    stats[ST_ELIGIBLE] = n_el;

    /* step 2: Morton order of the eligible patches (ties by patch index) */
    qsort(kp, (size_t)n_el, sizeof(kpair), cmp_kpair);

    /* step 3: fixed-point area prefix f(i) and its total f(N) */
    double unit = ldexp(ph * ph, -24);
    int64_t Q = 0;
    int* tri_of = (int*)malloc(sizeof(int) * (size_t)(n_el > 0 ? n_el : 1));
    for (int64_t j = 0; j < n_el; j++) {
        int g = kp[j].idx;
        int lo = 0, hi = s->T; /* triangle holding patch g: last t with patch_off[t] <= g */
        while (hi - lo > 1) { int mid = (lo + hi) / 2; if (patch_off[mid] <= g) lo = mid; else hi = mid; }
        tri_of[j] = lo;
        int n = level[lo];
        v3 cr = vcross(s->e1[lo], s->e2[lo]);
        double area = 0.5 * sqrt(vdot(cr, cr)) / ((double)n * (double)n);
        Q += llround(area / unit);
        F[j] = Q;
        sorted[j] = g;
        keys[j] = kp[j].key;
    }
    stats[ST_Q] = Q;
    int Keff = (Q > 0) ? K : 0;
    int n_far_t = n_far + (K - Keff);
    stats[ST_KEFF] = Keff;
    stats[ST_NFAR_TARGET] = n_far_t;
    if ((int64_t)Keff + n_far_t > cap) {
        free(level); free(kp); free(tri_of);
        return -1;
    }

    /* steps 4-5: K equal strata of [0, f(N)], midpoint target, inverse CDF;
     * one VPL per stratum placed by the square-root triangle formula with
     * Halton (2, 3) at index k + 1; its flux from eq. (2) with the area
     * D = f(N) / K that every VPL represents. */
    double D = ((double)Q * unit) / (double)K;
    int nv = 0;
    /* brightness = 1: eq. (2)'s light factor at every eligible patch's centroid */
    double* gpatch = NULL;
    if (brightness && Keff > 0) {
        gpatch = (double*)malloc(sizeof(double) * (size_t)n_el);
        for (int64_t j = 0; j < n_el; j++) {
            int g = kp[j].idx, t = tri_of[j], n = level[t];
            int a, b, down;
            local_to_ab(n, (int)(g - patch_off[t]), &a, &b, &down);
            v3 P[3];
            patch_verts(s, t, n, a, b, down, P);
            v3 c = mk((P[0].x + P[1].x + P[2].x) / 3.0, (P[0].y + P[1].y + P[2].y) / 3.0,
                      (P[0].z + P[1].z + P[2].z) / 3.0);
            gpatch[j] = light_factor(s, &L, c, s->n[t], t, eps);
        }
    }
    for (int kk = 0; kk < Keff; kk++) {
        /* stratum bounds B_k = floor(k f(N) / K) */
        int64_t Bk = (int64_t)(((__int128)kk * (__int128)Q) / (__int128)K);
        int64_t Bk1 = (int64_t)(((__int128)(kk + 1) * (__int128)Q) / (__int128)K);
        int64_t u;
        if (jitter) {
            int64_t len = Bk1 - Bk, off = 0;
            if (len > 0) {
                off = (int64_t)floor(oracle_halton(5, kk + 1) * (double)len);
                if (off > len - 1) off = len - 1;
            }
            u = Bk + off;
        } else {
            __int128 num = (__int128)(2 * (int64_t)kk + 1) * (__int128)Q;
            u = (int64_t)(num / (__int128)(2 * (int64_t)K));
        }
        int64_t lo = 0, hi = n_el; /* smallest j with F[j] > u */
        while (lo < hi) { int64_t mid = (lo + hi) / 2; if (F[mid] > u) hi = mid; else lo = mid + 1; }
        m[kk] = (int32_t)lo;
        int g = kp[lo].idx, t = tri_of[lo], n = level[t];
        int a, b, down;
        local_to_ab(n, (int)(g - patch_off[t]), &a, &b, &down);
        v3 P[3];
        patch_verts(s, t, n, a, b, down, P);
        double r1 = oracle_halton(2, kk + 1), r2 = oracle_halton(3, kk + 1);
        double sq = sqrt(r1);
        double w0 = 1.0 - sq, w1 = sq * (1.0 - r2), w2 = sq * r2;
        v3 y = mk(w0 * P[0].x + w1 * P[1].x + w2 * P[2].x, w0 * P[0].y + w1 * P[1].y + w2 * P[2].y,
                  w0 * P[0].z + w1 * P[1].z + w2 * P[2].z);
        v3 nk = s->n[t];
        vpl_pos[3 * nv] = y.x; vpl_pos[3 * nv + 1] = y.y; vpl_pos[3 * nv + 2] = y.z;
        vpl_nrm[3 * nv] = nk.x; vpl_nrm[3 * nv + 1] = nk.y; vpl_nrm[3 * nv + 2] = nk.z;
        if (!brightness) {
            double gsum = light_factor(s, &L, y, nk, t, eps);
            for (int c = 0; c < 3; c++) {
                double E = L.power[c] * gsum;
                double phi = (s->rho[3 * t + c] * E) * D;
                vpl_I[3 * nv + c] = phi / OR_PI;
            }
        } else {
            /* eq. (2) over the stratum's set of patches, in sorted order, each
             * with the part of its area inside [B_k, B_{k+1}) */
            double phi[3] = {0.0, 0.0, 0.0};
            int64_t j = 0, hj = n_el; /* first patch with F[j] > B_k */
            while (j < hj) { int64_t mid = (j + hj) / 2; if (F[mid] > Bk) hj = mid; else j = mid + 1; }
            for (; j < n_el; j++) {
                int64_t f0 = j > 0 ? F[j - 1] : 0, f1 = F[j];
                if (f0 >= Bk1) break;
                int64_t ov = (f1 < Bk1 ? f1 : Bk1) - (f0 > Bk ? f0 : Bk);
                if (ov <= 0) continue;
                int tj = tri_of[j];
                double A = (double)ov * unit;
                for (int c = 0; c < 3; c++) phi[c] += (s->rho[3 * tj + c] * (L.power[c] * gpatch[j])) * A;
            }
            for (int c = 0; c < 3; c++) vpl_I[3 * nv + c] = phi[c] / OR_PI;
        }
        vpl_tri[nv] = t;
        vpl_path[nv] = 0;
        vpl_bounce[nv] = 0;
        nv++;
    }

    /* steps 6-7: sparse quasi-random walk over the whole scene; hits on far
     * patches become VPLs, hits on near patches are discarded and the walk
     * continues.  Path i uses Halton index i with bases taken in prime
     * order as needed.  Stops with the path that brings the far count to
     * n_far_t; fluxes are then divided by the number of paths.  Variant
     * walk_near = 1 (not the paper's reading): only first-bounce near hits,
     * the light the patch VPLs stand for, are discarded; later near hits
     * become walk VPLs and count toward n_far_t; walk_near = 2: a near hit
     * ends its path. */
    int base_far = nv;
    int64_t path = 0;
    int nfar = 0;
    /* walk_schedule = 1: the number of paths and each bounce's path limit */
    double rb = 0.0;
    int64_t keller_n = 0, keller_t[3] = {0, 0, 0};
    if (walk_schedule) {
        rb = oracle_rho_bar((void*)s);
        double S = 0.0, r = 1.0;
        for (int j = 0; j < maxb; j++) { S += r; r *= rb; }
        keller_n = (int64_t)floor((double)n_far_t / S);
        if (keller_n > max_paths) { keller_n = max_paths; stats[ST_FLAGS] |= 1; }
        double rr = 1.0;
        for (int j = 0; j < maxb; j++) { keller_t[j] = (int64_t)floor(rr * (double)keller_n); rr *= rb; }
    }
    while (walk_schedule ? path < keller_n : nfar < n_far_t) {
        if (!walk_schedule && path >= max_paths) { stats[ST_FLAGS] |= 1; break; }
        path++;
        int dim = 0;
        v3 o, d;
        int ex = -1, skip_emit = 0;
        if (L.kind == 0) {
            double u1 = oracle_halton(PRIMES[dim], path), u2 = oracle_halton(PRIMES[dim + 1], path);
            dim += 2;
            double z = 1.0 - 2.0 * u1;
            double rr = sqrt(dmax(0.0, 1.0 - z * z));
            double phi = (2.0 * OR_PI) * u2;
            o = L.pos;
            d = mk(rr * cos(phi), rr * sin(phi), z);
        } else {
            double u1 = oracle_halton(PRIMES[0], path), u2 = oracle_halton(PRIMES[1], path);
            o = vadd(vadd(L.pos, vscl(L.eu, u1)), vscl(L.ev, u2));
            double u3 = oracle_halton(PRIMES[2], path), u4 = oracle_halton(PRIMES[3], path);
            d = cos_dir(L.nl, u3, u4);
            dim = 4;
            skip_emit = 1;
        }
        double flux[3] = {L.power[0], L.power[1], L.power[2]};
        for (int bnc = 1; bnc <= maxb && (walk_schedule || nfar < n_far_t); bnc++) {
            if (walk_schedule && path > keller_t[bnc - 1]) break;
            double tb, u, v;
            int t = closest(s, o, d, 0.0, INFINITY, ex, skip_emit, &tb, &u, &v);
            if (t < 0) break;                       /* miss */
            if (s->flags[t] & 1) break;             /* reached an emitter */
            if (!(vdot(d, s->n[t]) < 0.0)) break;   /* back side of a one-sided face */
            for (int c = 0; c < 3; c++) {
                flux[c] = flux[c] * s->rho[3 * t + c];
                if (walk_schedule && bnc >= 2) flux[c] = flux[c] / rb;
            }
            v3 y = vadd(vadd(s->A[t], vscl(s->e1[t], u)), vscl(s->e2[t], v));
            /* the patch of the hit point, from its barycentric coordinates */
            int n = level[t];
            double U = u * (double)n, V = v * (double)n;
            int a = (int)floor(U), b = (int)floor(V);
            if (a < 0) a = 0;
            if (b < 0) b = 0;
            if (a > n - 1) a = n - 1;
            if (b > n - 1) b = n - 1;
            if (a + b > n - 1) a = n - 1 - b;
            int down = (a + b <= n - 2) && ((U - (double)a) + (V - (double)b) > 1.0);
            int64_t g = patch_off[t] + (int64_t)b * (2 * n - b) + 2 * a + down;
            if (!(pflags[g] & 1) || (walk_near == 1 && bnc >= 2)) {
                if (nv >= cap) { free(level); free(kp); free(tri_of); free(gpatch); return -1; }
                vpl_pos[3 * nv] = y.x; vpl_pos[3 * nv + 1] = y.y; vpl_pos[3 * nv + 2] = y.z;
                vpl_nrm[3 * nv] = s->n[t].x; vpl_nrm[3 * nv + 1] = s->n[t].y; vpl_nrm[3 * nv + 2] = s->n[t].z;
                for (int c = 0; c < 3; c++) vpl_I[3 * nv + c] = flux[c]; /* normalised below */
                vpl_tri[nv] = t;
                vpl_path[nv] = (int32_t)path;
                vpl_bounce[nv] = bnc;
                stats[ST_B1 + bnc - 1]++;
                nv++;
                nfar++;
            } else {
                stats[ST_NEAR_DISCARDED]++;
                if (walk_near == 2) break; /* the near hit ends the path */
            }
            if (bnc == maxb) break;
            double s1 = oracle_halton(PRIMES[dim], path), s2 = oracle_halton(PRIMES[dim + 1], path);
            dim += 2;
            o = y;
            d = cos_dir(s->n[t], s1, s2);
            ex = t;
            skip_emit = 0;
        }
    }
    stats[ST_NPATHS] = path;
    stats[ST_NFAR] = nfar;
    for (int i = base_far; i < nv; i++)
        for (int c = 0; c < 3; c++) {
            double phi = vpl_I[3 * i + c] / (double)path;
            vpl_I[3 * i + c] = phi / OR_PI;
        }
    free(level);
    free(kp);
    free(tri_of);
    free(gpatch);
    return nv;
}

/* Morton key of integer cells, exposed for the tests. */
uint32_t oracle_morton30(int cx, int cy, int cz) { return morton30(cx, cy, cz); }

int oracle_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
