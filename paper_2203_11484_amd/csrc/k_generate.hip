// FP64 kernels of the hybrid VPL generation (Section "Close-Range VPL
// Sampling"), compiled with -ffp-contract=off.
//
//   1. refine every one-sided face into patches with edges <= h
//   2. classify patches: near = centroid in the view frustum and closer than
//      d_near; eligible = near and facing the light
//   3. order eligible patches by (Morton key of the centroid, patch index)
//   4. fixed-point area prefix f(i); K strata of [0, f(N)] with midpoint
//      targets (or, jitter = 1, targets jittered inside the integer stratum
//      bounds B_k = floor(k f(N) / K)); inverse CDF picks the patch of each VPL
//   5. place the VPL with the square-root triangle formula at Halton
//      (2, 3)(k + 1), brightness from eq. (2) with area f(N)/K (or,
//      brightness = 1, eq. (2) summed over the stratum's patches at their
//      centroids, each with its area inside [B_k, B_{k+1}))
//   6. sparse quasi-random walk from the light; hits on far patches become
//      VPLs, hits on near patches are discarded (walk_near = 1: only at the
//      first bounce; walk_near = 2: the near hit ends its path), until n_far
//      VPLs exist
//
// Integer outcomes (levels, flags, order, strata, hit triangles, path
// counts) are decided in FP64 with a fixed operation order so that a plain
// CPU evaluation of the same definitions reproduces them exactly.
#include "vplg_impl.h"

namespace vplg {

namespace {

constexpr double kPi = 3.14159265358979323846;
constexpr int GB = 256;

// The first eight primes: Halton bases taken in order as a path needs them.
__device__ __forceinline__ int prime(int i)
{
    switch (i) {
    case 0: return 2;
    case 1: return 3;
    case 2: return 5;
    case 3: return 7;
    case 4: return 11;
    case 5: return 13;
    case 6: return 17;
    default: return 19;
    }
}

struct d3 {
    double x, y, z;
};
__device__ __forceinline__ d3 mk(double x, double y, double z) { return d3{x, y, z}; }
__device__ __forceinline__ d3 add(d3 a, d3 b) { return mk(a.x + b.x, a.y + b.y, a.z + b.z); }
__device__ __forceinline__ d3 sub(d3 a, d3 b) { return mk(a.x - b.x, a.y - b.y, a.z - b.z); }
__device__ __forceinline__ d3 scl(d3 a, double s) { return mk(a.x * s, a.y * s, a.z * s); }
__device__ __forceinline__ double dot(d3 a, d3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
__device__ __forceinline__ d3 cross(d3 a, d3 b)
{
    return mk(a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x);
}
__device__ __forceinline__ d3 norm(d3 a)
{
    double l = sqrt(dot(a, a));
    return mk(a.x / l, a.y / l, a.z / l);
}
__device__ __forceinline__ double dmax(double a, double b) { return a > b ? a : b; }
__device__ __forceinline__ d3 ldf(const float* p) { return mk((double)p[0], (double)p[1], (double)p[2]); }
__device__ __forceinline__ d3 vA(const DevScene& s, int t) { return ldf(s.xyz + 9 * t); }
__device__ __forceinline__ d3 vB(const DevScene& s, int t) { return ldf(s.xyz + 9 * t + 3); }
__device__ __forceinline__ d3 vC(const DevScene& s, int t) { return ldf(s.xyz + 9 * t + 6); }

// Radical inverse of i in base b as the exact ratio num / b^m.
__device__ double halton(int b, long long i)
{
    unsigned long long num = 0, den = 1, q = (unsigned long long)i, ub = (unsigned long long)b;
    while (q > 0) {
        num = num * ub + q % ub;
        den *= ub;
        q /= ub;
    }
    return (double)num / (double)den;
}

__device__ int patch_level(const DevScene& s, int t, double h)
{
    d3 A = vA(s, t), B = vB(s, t), C = vC(s, t);
    d3 a = sub(B, A), b = sub(C, B), c = sub(A, C);
    double m2 = dmax(dmax(dot(a, a), dot(b, b)), dot(c, c));
    int n = (int)floor(sqrt(m2) / h) - 1;
    if (n < 1) n = 1;
    while (((double)n * h) * ((double)n * h) < m2) n++;
    return n;
}

__device__ __forceinline__ d3 grid_pt(d3 A, d3 e1, d3 e2, int n, int a, int b)
{
    return add(add(A, scl(e1, (double)a / (double)n)), scl(e2, (double)b / (double)n));
}

__device__ __forceinline__ void local_to_ab(int n, int local, int* a, int* b, int* down)
{
    int r = 0;
    while ((long long)(r + 1) * (2 * n - (r + 1)) <= local) r++;
    int rem = local - r * (2 * n - r);
    *b = r;
    *a = rem / 2;
    *down = rem & 1;
}

__device__ void patch_verts(d3 A, d3 e1, d3 e2, int n, int a, int b, int down, d3* P)
{
    if (!down) {
        P[0] = grid_pt(A, e1, e2, n, a, b); P[1] = grid_pt(A, e1, e2, n, a + 1, b); P[2] = grid_pt(A, e1, e2, n, a, b + 1);
    } else {
        P[0] = grid_pt(A, e1, e2, n, a + 1, b); P[1] = grid_pt(A, e1, e2, n, a + 1, b + 1);
        P[2] = grid_pt(A, e1, e2, n, a, b + 1);
    }
}

struct Cam64 {
    d3 eye, f, r, u;
    double th, tx;
};

__device__ __forceinline__ Cam64 cam64(const CamBasis& c)
{
    Cam64 k;
    k.eye = mk(c.eye[0], c.eye[1], c.eye[2]);
    k.f = mk(c.f[0], c.f[1], c.f[2]);
    k.r = mk(c.r[0], c.r[1], c.r[2]);
    k.u = mk(c.u[0], c.u[1], c.u[2]);
    k.th = c.th;
    k.tx = c.tx;
    return k;
}

__device__ __forceinline__ bool is_near(const Cam64& k, d3 c, double dn)
{
    d3 v = sub(c, k.eye);
    double z = dot(v, k.f);
    if (!(z > 0.0)) return false;
    if (!(fabs(dot(v, k.r)) <= z * k.tx)) return false;
    if (!(fabs(dot(v, k.u)) <= z * k.th)) return false;
    return dot(v, v) < dn * dn;
}

struct Light64 {
    int kind;
    d3 pos, eu, ev, nl, lc;
    double power[3];
};

__device__ __forceinline__ Light64 light64(const DevLight& L)
{
    Light64 o;
    o.kind = L.kind;
    o.pos = mk(L.pos[0], L.pos[1], L.pos[2]);
    o.eu = mk(L.eu[0], L.eu[1], L.eu[2]);
    o.ev = mk(L.ev[0], L.ev[1], L.ev[2]);
    for (int c = 0; c < 3; ++c) o.power[c] = (double)L.power[c];
    if (o.kind == 1) {
        o.nl = norm(cross(o.eu, o.ev));
        o.lc = add(add(o.pos, scl(o.eu, 0.5)), scl(o.ev, 0.5));
    } else {
        o.nl = mk(0, 0, 0);
        o.lc = o.pos;
    }
    return o;
}

__device__ __forceinline__ unsigned morton30(int cx, int cy, int cz)
{
    unsigned key = 0;
    for (int b = 0; b < 10; ++b) {
        key |= (unsigned)((cx >> b) & 1) << (3 * b);
        key |= (unsigned)((cy >> b) & 1) << (3 * b + 1);
        key |= (unsigned)((cz >> b) & 1) << (3 * b + 2);
    }
    return key;
}

__device__ __forceinline__ int cell_of(double c, double lo, double h)
{
    double f = floor((c - lo) / h);
    if (f < 0.0) f = 0.0;
    if (f > 1023.0) f = 1023.0;
    return (int)f;
}

// ---------------------------------------------------------------------------
// FP64 ray casting over the float BVH (boxes are padded outward by the
// builder, so a double slab test never drops a box the exact ray touches).
// ---------------------------------------------------------------------------

// Moller-Trumbore on the original float vertices, in FP64, fixed order.
__device__ __forceinline__ bool tri64(const DevScene& s, int t, d3 o, d3 d, double* tt, double* uu, double* vv)
{
    d3 A = vA(s, t);
    d3 e1 = sub(vB(s, t), A), e2 = sub(vC(s, t), A);
    d3 pvec = cross(d, e2);
    double det = dot(e1, pvec);
    if (det == 0.0) return false;
    double inv = 1.0 / det;
    d3 tvec = sub(o, A);
    double u = dot(tvec, pvec) * inv;
    if (u < 0.0 || u > 1.0) return false;
    d3 qvec = cross(tvec, e1);
    double v = dot(d, qvec) * inv;
    if (v < 0.0 || u + v > 1.0) return false;
    *tt = dot(e2, qvec) * inv;
    *uu = u;
    *vv = v;
    return true;
}

constexpr int kStack64 = kStack + 2;
// The FP64 traversals keep their stacks in LDS, [entry][thread] for kGenBlock
// threads (one per lane: entries of a lane are kGenBlock words apart, so the
// lanes of a wave hit distinct banks).  A private array indexed at run time
// would live in scratch memory, with a memory round trip per push and pop.
constexpr int kGenBlock = 64;
struct LdsStack {
    int* base;  // &stack[0][thread]
    __device__ __forceinline__ int& operator[](int i) const { return base[i * kGenBlock]; }
};
#define VPLG_LDS_STACK(name)                                   \
    __shared__ int name##_mem[kStack64 * kGenBlock];          \
    const LdsStack name{name##_mem + threadIdx.x}

// Per-ray inverse direction for the FP64 slab tests; an axis with a zero
// component is flagged and tested by containment instead.
struct Inv64 {
    double o[3], inv[3];
    bool zero[3];
};

__device__ __forceinline__ Inv64 inv64(d3 o, d3 d)
{
    Inv64 r;
    const double oo[3] = {o.x, o.y, o.z}, dd[3] = {d.x, d.y, d.z};
    for (int k = 0; k < 3; ++k) {
        r.o[k] = oo[k];
        r.zero[k] = dd[k] == 0.0;
        r.inv[k] = r.zero[k] ? 0.0 : 1.0 / dd[k];
    }
    return r;
}

// Entry parameter of the ray into the box within (tmin, tmax), or +inf if
// it misses.  Plane distances are (plane - o) * (1 / d): within an ulp of
// the quotient, far inside the boxes' outward padding, so no box that holds
// a hit inside (tmin, tmax) is culled and the hit found is the same.
__device__ __forceinline__ double slab64(double lx, double hx, double ly, double hy, double lz, double hz,
                                         const Inv64& r, double tmin, double tmax)
{
    const double lo[3] = {lx, ly, lz}, hi[3] = {hx, hy, hz};
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        if (r.zero[k]) {
            if (r.o[k] < lo[k] || r.o[k] > hi[k]) return __builtin_inf();
            continue;
        }
        double t0 = (lo[k] - r.o[k]) * r.inv[k], t1 = (hi[k] - r.o[k]) * r.inv[k];
        if (t0 > t1) { double tmp = t0; t0 = t1; t1 = tmp; }
        tmin = t0 > tmin ? t0 : tmin;
        tmax = t1 < tmax ? t1 : tmax;
        if (tmin > tmax) return __builtin_inf();
    }
    return tmin;
}

// Visibility (segment, s in (eps, 1 - eps), host triangles tx / ty skipped).
__device__ bool visible64(const DevScene& s, d3 x, int tx, d3 y, int ty, double eps, LdsStack stack)
{
    d3 d = sub(y, x);
    double lo = eps, hi = 1.0 - eps;
    const Inv64 ri = inv64(x, d);
    int sp = 0;
    stack[sp++] = 0;
    while (sp > 0) {
        int node = stack[--sp];
        const float4* n = s.nodes + 4 * node;
        float4 n0 = n[0], n1 = n[1], n2 = n[2], n3f = n[3];
        int c[2] = {__float_as_int(n3f.x), __float_as_int(n3f.y)};
        const int kk = __float_as_int(n3f.z);
        int k[2] = {kk & 0xffff, kk >> 16};
        for (int ch = 0; ch < 2; ++ch) {
            const double e = ch == 0 ? slab64(n0.x, n0.y, n0.z, n0.w, n2.x, n2.y, ri, lo, hi)
                                     : slab64(n1.x, n1.y, n1.z, n1.w, n2.z, n2.w, ri, lo, hi);
            if (!(e < __builtin_inf())) continue;
            if (k[ch] > 0) {
                for (int i = c[ch]; i < c[ch] + k[ch]; ++i) {
                    int t = __float_as_int(s.tris[kTriStride * i].w);
                    double tt, u, v;
                    if (t == tx || t == ty) continue;
                    if (tri64(s, t, x, d, &tt, &u, &v) && tt > lo && tt < hi) return false;
                }
            } else {
                stack[sp++] = c[ch];
            }
        }
    }
    return true;
}

// Closest hit with t in (tmin, inf), ties to the smaller triangle index;
// triangle ex and (if skip_emit) emitters are skipped.
__device__ int closest64(const DevScene& s, d3 o, d3 d, double tmin, int ex, bool skip_emit, double* tb, double* ub,
                         double* vb, LdsStack stack)
{
    int best = -1;
    double bt = __builtin_inf(), bu = 0, bv = 0;
    const Inv64 ri = inv64(o, d);
    int sp = 0;
    stack[sp++] = 0;
    while (sp > 0) {
        int node = stack[--sp];
        const float4* n = s.nodes + 4 * node;
        float4 n0 = n[0], n1 = n[1], n2 = n[2], n3f = n[3];
        const int c[2] = {__float_as_int(n3f.x), __float_as_int(n3f.y)};
        const int kk = __float_as_int(n3f.z);
        const int k[2] = {kk & 0xffff, kk >> 16};
        double e[2] = {slab64(n0.x, n0.y, n0.z, n0.w, n2.x, n2.y, ri, tmin, bt),
                       slab64(n1.x, n1.y, n1.z, n1.w, n2.z, n2.w, ri, tmin, bt)};
        // leaf children first (their hits shrink bt), then the inner
        // children, the nearer one on top of the stack; a child is entered
        // iff the ray meets its box within (tmin, bt] (a miss is +inf)
        for (int ch = 0; ch < 2; ++ch) {
            if (k[ch] == 0 || !(e[ch] < __builtin_inf() && e[ch] <= bt)) continue;
            for (int i = c[ch]; i < c[ch] + k[ch]; ++i) {
                int t = __float_as_int(s.tris[kTriStride * i].w);
                double tt, u, v;
                if (t == ex || (skip_emit && (s.flags[t] & 1))) continue;
                if (tri64(s, t, o, d, &tt, &u, &v) && tt > tmin) {
                    if (best < 0 || tt < bt || (tt == bt && t < best)) { best = t; bt = tt; bu = u; bv = v; }
                }
            }
        }
        const bool in0 = k[0] == 0 && e[0] < __builtin_inf() && e[0] <= bt;
        const bool in1 = k[1] == 0 && e[1] < __builtin_inf() && e[1] <= bt;
        if (in0 && in1) {
            const bool near0 = e[0] <= e[1];
            stack[sp++] = near0 ? c[1] : c[0];
            stack[sp++] = near0 ? c[0] : c[1];
        } else if (in0) {
            stack[sp++] = c[0];
        } else if (in1) {
            stack[sp++] = c[1];
        }
    }
    *tb = bt; *ub = bu; *vb = bv;
    return best;
}

// Duff et al. 2017 orthonormal basis around n; returns x b1 + y b2 + z n.
__device__ __forceinline__ d3 onb_dir(d3 n, double x, double y, double z)
{
    double sign = copysign(1.0, n.z);
    double a = -1.0 / (sign + n.z);
    double b = n.x * n.y * a;
    d3 b1 = mk(1.0 + sign * n.x * n.x * a, sign * b, -sign * n.x);
    d3 b2 = mk(b, sign + n.y * n.y * a, -n.y);
    return mk(x * b1.x + y * b2.x + z * n.x, x * b1.y + y * b2.y + z * n.y, x * b1.z + y * b2.z + z * n.z);
}

__device__ __forceinline__ d3 cos_dir(d3 n, double u1, double u2)
{
    double r = sqrt(u1);
    double ph = (2.0 * kPi) * u2;
    return onb_dir(n, r * cos(ph), r * sin(ph), sqrt(dmax(0.0, 1.0 - u1)));
}

// ---------------------------------------------------------------------------
// kernels
// ---------------------------------------------------------------------------

__global__ void k_patch_levels(DevScene s, double h, int32_t* level, long long* counts)
{
    int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= s.n_tris) return;
    int n = patch_level(s, t, h);
    level[t] = n;
    counts[t] = (long long)n * n;
}

__device__ __forceinline__ int tri_of_patch(const long long* off, int T, long long g)
{
    int lo = 0, hi = T;  // last t with off[t] <= g
    while (hi - lo > 1) {
        int mid = (lo + hi) >> 1;
        if (off[mid] <= g) lo = mid; else hi = mid;
    }
    return lo;
}

// Flags and sort keys of every patch; non-eligible patches sort last.
__global__ void k_classify(DevScene s, CamBasis cb, DevLight dl, GenParams p, GenBuffers b)
{
    long long g = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    __shared__ int s_near, s_el;
    __shared__ unsigned long long s_base;
    if (threadIdx.x == 0) { s_near = 0; s_el = 0; }
    __syncthreads();
    unsigned long long key = ~0ull;
    int pos = -1;  // this patch's place among the block's eligible patches
    if (g < b.n_patches) {
        int t = tri_of_patch(b.patch_off, s.n_tris, g);
        int n = b.level[t];
        int a, bb, down;
        local_to_ab(n, (int)(g - b.patch_off[t]), &a, &bb, &down);
        d3 A = vA(s, t);
        d3 e1 = sub(vB(s, t), A), e2 = sub(vC(s, t), A);
        d3 P[3];
        patch_verts(A, e1, e2, n, a, bb, down, P);
        d3 c = mk((P[0].x + P[1].x + P[2].x) / 3.0, (P[0].y + P[1].y + P[2].y) / 3.0,
                  (P[0].z + P[1].z + P[2].z) / 3.0);
        Cam64 k = cam64(cb);
        Light64 L = light64(dl);
        uint8_t fl = 0;
        if (!(s.flags[t] & 1) && is_near(k, c, p.d_near)) {
            fl |= 1;
            d3 nt = norm(cross(e1, e2));
            bool el = dot(nt, sub(L.lc, c)) > 0.0;
            if (L.kind == 1) el = el && (dot(L.nl, sub(c, L.lc)) > 0.0);
            if (el) {
                fl |= 2;
                double lo[3] = {(double)s.lo[0], (double)s.lo[1], (double)s.lo[2]};
                unsigned m = morton30(cell_of(c.x, lo[0], p.patch_h), cell_of(c.y, lo[1], p.patch_h),
                                      cell_of(c.z, lo[2], p.patch_h));
                key = ((unsigned long long)m << 32) | (unsigned long long)g;
            }
        }
        b.pflags[g] = fl;
        if (fl & 1) atomicAdd(&s_near, 1);
        if (fl & 2) pos = atomicAdd(&s_el, 1);
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        if (s_near) atomicAdd((unsigned long long*)&b.state->n_near, (unsigned long long)s_near);
        s_base = s_el ? atomicAdd((unsigned long long*)&b.state->n_eligible, (unsigned long long)s_el) : 0ull;
    }
    __syncthreads();
    // eligible keys go to the front of the sort buffer, in any order: the
    // (key, patch) pairs are unique, so their sorted order is fixed
    if (pos >= 0) b.sortbuf[s_base + pos] = key;
}

constexpr int kLocal = 2048;  // elements per workgroup in the LDS stages

// The sort runs on the front of the buffer that holds the eligible keys: the
// next power of two >= max(n_eligible, kLocal) elements (the rest are all-ones
// keys that stay in place).  Passes of a larger level, and elements past it,
// have nothing to do.
__device__ __forceinline__ long long sort_extent(const GenState* st)
{
    const long long ne = st->n_eligible;
    long long m = kLocal;
    while (m < ne) m <<= 1;
    return m;
}

// Bitonic sort (ascending) of a power-of-two array of unique 64-bit keys.
__global__ void k_bitonic_global(unsigned long long* a, long long n, long long j, long long k, const GenState* st)
{
    long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const long long m = sort_extent(st);
    if (i >= n || i >= m || k > m) return;
    long long l = i ^ j;
    if (l > i) {
        unsigned long long x = a[i], y = a[l];
        bool up = (i & k) == 0;
        if ((x > y) == up) { a[i] = y; a[l] = x; }
    }
}

// All stages j < kLocal of level k (k <= kLocal: the whole local sort up to k).
__global__ __launch_bounds__(1024) void k_bitonic_local(unsigned long long* a, long long n, long long k_from,
                                                        long long k_to, long long j_from, const GenState* st)
{
    __shared__ unsigned long long s[kLocal];
    long long base = (long long)blockIdx.x * kLocal;
    const long long m = sort_extent(st);
    if (base >= m || k_from > m) return;  // uniform over the workgroup
    for (int i = threadIdx.x; i < kLocal; i += blockDim.x) s[i] = a[base + i];
    __syncthreads();
    for (long long k = k_from; k <= k_to; k <<= 1) {
        for (long long j = (k == k_from ? j_from : k >> 1); j > 0; j >>= 1) {
            for (int i = threadIdx.x; i < kLocal; i += blockDim.x) {
                int l = i ^ (int)j;
                if (l > i) {
                    long long gi = base + i;
                    unsigned long long x = s[i], y = s[l];
                    bool up = (gi & k) == 0;
                    if ((x > y) == up) { s[i] = y; s[l] = x; }
                }
            }
            __syncthreads();
        }
    }
    for (int i = threadIdx.x; i < kLocal; i += blockDim.x) a[base + i] = s[i];
}

// Sorted eligible patches, their keys and fixed-point areas q = llround(area / unit).
__global__ void k_sorted_areas(DevScene s, GenParams p, GenBuffers b, long long* q)
{
    long long j = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= b.n_patches) return;
    long long ne = b.state->n_eligible;
    if (j >= ne) { q[j] = 0; return; }
    unsigned long long key = b.sortbuf[j];
    int g = (int)(key & 0xffffffffull);
    b.sorted[j] = g;
    b.keys[j] = (uint32_t)(key >> 32);
    int t = tri_of_patch(b.patch_off, s.n_tris, g);
    int n = b.level[t];
    d3 A = vA(s, t);
    d3 e1 = sub(vB(s, t), A), e2 = sub(vC(s, t), A);
    d3 cr = cross(e1, e2);
    double area = 0.5 * sqrt(dot(cr, cr)) / ((double)n * (double)n);
    double unit = (p.patch_h * p.patch_h) * 0x1p-24;
    q[j] = (long long)round(area / unit);
}

// Eq. (2)'s light factor at point y (normal nk, on triangle t) per unit
// power: V cos / (4 pi r^2) for the point light, or the mean over the 16
// quad cells of V cos_l cos / (pi r^2).
__device__ double light_factor64(const DevScene& s, const Light64& L, d3 y, d3 nk, int t, double t_eps,
                                 LdsStack stk)
{
    double gsum = 0.0;
    if (L.kind == 0) {
        d3 w = sub(L.pos, y);
        double r2w = dot(w, w);
        double r = sqrt(r2w);
        double ck = dot(nk, w) / r;
        if (ck > 0.0 && visible64(s, y, t, L.pos, -1, t_eps, stk)) gsum = ck / ((4.0 * kPi) * r2w);
    } else {
        for (int j = 0; j < 16; ++j) {
            d3 lj = add(add(L.pos, scl(L.eu, ((double)(j % 4) + 0.5) / 4.0)), scl(L.ev, ((double)(j / 4) + 0.5) / 4.0));
            d3 w = sub(lj, y);
            double r2w = dot(w, w);
            double r = sqrt(r2w);
            double cl = -dot(L.nl, w) / r;
            double ck = dot(nk, w) / r;
            if (cl > 0.0 && ck > 0.0 && visible64(s, y, t, lj, -1, t_eps, stk)) gsum += (cl * ck) / (kPi * r2w);
        }
        gsum = gsum / 16.0;
    }
    return gsum;
}

// The term of light sample j in light_factor64's sum (0 when it does not
// count): the lanes of a group evaluate one sample each, and the group's
// first lane adds them in sample order, which reproduces the sequential sum
// bit for bit (adding an exact 0 leaves a sum unchanged).
__device__ double light_term64(const DevScene& s, const Light64& L, d3 y, d3 nk, int t, double t_eps, int j,
                               LdsStack stk)
{
    if (L.kind == 0) {
        d3 w = sub(L.pos, y);
        double r2w = dot(w, w);
        double r = sqrt(r2w);
        double ck = dot(nk, w) / r;
        return ck > 0.0 && visible64(s, y, t, L.pos, -1, t_eps, stk) ? ck / ((4.0 * kPi) * r2w) : 0.0;
    }
    d3 lj = add(add(L.pos, scl(L.eu, ((double)(j % 4) + 0.5) / 4.0)), scl(L.ev, ((double)(j / 4) + 0.5) / 4.0));
    d3 w = sub(lj, y);
    double r2w = dot(w, w);
    double r = sqrt(r2w);
    double cl = -dot(L.nl, w) / r;
    double ck = dot(nk, w) / r;
    return cl > 0.0 && ck > 0.0 && visible64(s, y, t, lj, -1, t_eps, stk) ? (cl * ck) / (kPi * r2w) : 0.0;
}

// Light factor of the item of a group of S lanes (S = 16: one quad-light
// sample per lane; S = 1: the whole sum in one lane).  Every lane of the block
// must call it (a barrier); the result is valid in the group's first lane.
template <int S>
__device__ double light_factor_group(const DevScene& s, const Light64& L, d3 y, d3 nk, int t, double t_eps, bool live,
                                     double* s_term, LdsStack stk)
{
    if constexpr (S == 1) {
        return live ? light_factor64(s, L, y, nk, t, t_eps, stk) : 0.0;
    } else {
        const int sub = threadIdx.x % S;
        s_term[threadIdx.x] = live ? light_term64(s, L, y, nk, t, t_eps, sub, stk) : 0.0;
        __syncthreads();
        double gsum = 0.0;
        if (sub == 0)
            for (int i = 0; i < S; ++i) gsum += s_term[threadIdx.x + i];
        return gsum / 16.0;
    }
}

// brightness = 1: the light factor at the centroid of every eligible patch,
// in sorted order (runs after k_sorted_areas: patch_g reuses the sort buffer).
template <int S>
__global__ __launch_bounds__(kGenBlock) void k_patch_light(DevScene s, DevLight dl, GenParams p, GenBuffers b)
{
    VPLG_LDS_STACK(stk);
    __shared__ double s_term[kGenBlock];
    const long long j = (long long)blockIdx.x * (kGenBlock / S) + threadIdx.x / S;
    const bool live = j < b.state->n_eligible;
    d3 c = mk(0.0, 0.0, 0.0), nk = mk(0.0, 0.0, 1.0);
    int t = 0;
    if (live) {
        int g = b.sorted[j];
        t = tri_of_patch(b.patch_off, s.n_tris, g);
        int n = b.level[t];
        int a, bb, down;
        local_to_ab(n, (int)(g - b.patch_off[t]), &a, &bb, &down);
        d3 A = vA(s, t);
        d3 e1 = sub(vB(s, t), A), e2 = sub(vC(s, t), A);
        d3 P[3];
        patch_verts(A, e1, e2, n, a, bb, down, P);
        c = mk((P[0].x + P[1].x + P[2].x) / 3.0, (P[0].y + P[1].y + P[2].y) / 3.0, (P[0].z + P[1].z + P[2].z) / 3.0);
        nk = norm(cross(e1, e2));
    }
    const double gsum = light_factor_group<S>(s, light64(dl), c, nk, t, p.t_eps, live, s_term, stk);
    if (live && threadIdx.x % S == 0) b.patch_g[j] = gsum;
}

__global__ void k_strata_state(GenParams p, GenBuffers b, double rho_bar)
{
    // q_total, k_eff and the far target, once the prefix is known.
    long long ne = b.state->n_eligible;
    long long Q = ne > 0 ? b.F[ne - 1] : 0;
    b.state->q_total = Q;
    b.state->k_eff = Q > 0 ? p.k_near : 0;
    b.state->n_far_target = p.n_far + (Q > 0 ? 0 : p.k_near);
    // (2K + 1) Q must fit in int64 for the midpoint targets
    if (Q > 0 && Q > 0x7fffffffffffffffll / (2ll * p.k_near + 1)) b.state->flags |= 2;
    if (p.walk_schedule) {
        // Keller's schedule: N = floor(target / sum_j rb^j) paths, bounce b
        // open to paths i <= floor(rb^(b-1) N)
        double S = 0.0, r = 1.0;
        for (int j = 0; j < p.max_bounces; ++j) { S += r; r *= rho_bar; }
        long long N = (long long)floor((double)b.state->n_far_target / S);
        if (N > p.max_paths) { N = p.max_paths; b.state->flags |= 1; }
        b.state->keller_n = N;
        double rr = 1.0;
        for (int j = 0; j < p.max_bounces; ++j) { b.state->keller_t[j] = (long long)floor(rr * (double)N); rr *= rho_bar; }
    }
    // a zero far target needs no path at all
    if (b.state->n_far_target == 0) {
        b.state->walk_done = 1;
        b.state->n_far = 0;
        b.state->n_paths = 0;
    }
}

// One VPL per stratum: midpoint target, inverse CDF, placement, eq. (2).
// (block `blk` of the strata's blocks; every lane of the block must call it)
template <int S>
__device__ __forceinline__ void strata_block(const DevScene& s, const DevLight& dl, const GenParams& p, const GenBuffers& b,
                             const DevVpls& v, int blk, LdsStack stk, double* s_term)
{
    // S lanes per stratum (one quad-light sample each), else one
    const int kk = blk * (kGenBlock / S) + threadIdx.x / S;
    const bool live = kk < b.state->k_eff && !(b.state->flags & 2);
    const bool lead = threadIdx.x % S == 0;
    long long Q = 0, ne = 0, Bk = 0, Bk1 = 0;
    const long long K = p.k_near;
    d3 y = mk(0.0, 0.0, 0.0), nk = mk(0.0, 0.0, 1.0);
    int t = 0;
    if (live) {
        Q = b.state->q_total;
        ne = b.state->n_eligible;
        // stratum bounds B_k = floor(k f(N) / K) (k Q fits: (2K + 1) Q does)
        Bk = ((long long)kk * Q) / K;
        Bk1 = ((long long)(kk + 1) * Q) / K;
        long long u;
        if (p.jitter) {
            const long long len = Bk1 - Bk;
            long long off = 0;
            if (len > 0) {
                off = (long long)floor(halton(5, kk + 1) * (double)len);
                if (off > len - 1) off = len - 1;
            }
            u = Bk + off;
        } else {
            u = ((2 * (long long)kk + 1) * Q) / (2 * K);
        }
        long long lo = 0, hi = ne;  // smallest j with F[j] > u
        while (lo < hi) {
            long long mid = (lo + hi) >> 1;
            if (b.F[mid] > u) hi = mid; else lo = mid + 1;
        }
        if (lead) b.strata[kk] = (int32_t)lo;
        int g = b.sorted[lo];
        t = tri_of_patch(b.patch_off, s.n_tris, g);
        int n = b.level[t];
        int a, bb, down;
        local_to_ab(n, (int)(g - b.patch_off[t]), &a, &bb, &down);
        d3 A = vA(s, t);
        d3 e1 = sub(vB(s, t), A), e2 = sub(vC(s, t), A);
        d3 P[3];
        patch_verts(A, e1, e2, n, a, bb, down, P);
        double r1 = halton(2, kk + 1), r2 = halton(3, kk + 1);
        double sq = sqrt(r1);
        double w0 = 1.0 - sq, w1 = sq * (1.0 - r2), w2 = sq * r2;
        y = mk(w0 * P[0].x + w1 * P[1].x + w2 * P[2].x, w0 * P[0].y + w1 * P[1].y + w2 * P[2].y,
               w0 * P[0].z + w1 * P[1].z + w2 * P[2].z);
        nk = norm(cross(e1, e2));
    }
    Light64 L = light64(dl);
    // eq. (2)'s light factor at the VPL's point (every lane of the block takes part)
    const double gsum = p.brightness ? 0.0 : light_factor_group<S>(s, L, y, nk, t, p.t_eps, live, s_term, stk);
    if (!live || !lead) return;
    v.px[kk] = (float)y.x; v.py[kk] = (float)y.y; v.pz[kk] = (float)y.z;
    v.nx[kk] = (float)nk.x; v.ny[kk] = (float)nk.y; v.nz[kk] = (float)nk.z;
    float* outs[3] = {v.ir, v.ig, v.ib};
    const double unit = (p.patch_h * p.patch_h) * 0x1p-24;
    if (!p.brightness) {
        double D = ((double)Q * unit) / (double)K;
        for (int c = 0; c < 3; ++c) {
            double E = L.power[c] * gsum;
            double phi = ((double)s.albedo[3 * t + c] * E) * D;
            outs[c][kk] = (float)(phi / kPi);
        }
    } else {
        // eq. (2) over the stratum's patches in sorted order, each with the
        // part of its fixed-point area inside [B_k, B_{k+1})
        double phi[3] = {0.0, 0.0, 0.0};
        long long j = 0, hj = ne;  // first patch with F[j] > B_k
        while (j < hj) {
            long long mid = (j + hj) >> 1;
            if (b.F[mid] > Bk) hj = mid; else j = mid + 1;
        }
        for (; j < ne; ++j) {
            const long long f0 = j > 0 ? b.F[j - 1] : 0, f1 = b.F[j];
            if (f0 >= Bk1) break;
            const long long ov = (f1 < Bk1 ? f1 : Bk1) - (f0 > Bk ? f0 : Bk);
            if (ov <= 0) continue;
            const int tj = tri_of_patch(b.patch_off, s.n_tris, b.sorted[j]);
            const double A = (double)ov * unit;
            const double gj = b.patch_g[j];
            for (int c = 0; c < 3; ++c) phi[c] += ((double)s.albedo[3 * tj + c] * (L.power[c] * gj)) * A;
        }
        for (int c = 0; c < 3; ++c) outs[c][kk] = (float)(phi[c] / kPi);
    }
    v.tri[kk] = t;
    b.vpl_path[kk] = 0;
    b.vpl_bounce[kk] = 0;
}

// One thread per walk path of the batch [start + 1, start + batch].
// Paths per 64-lane block of the walk.  A wave lasts as long as its slowest
// path, so 16 paths per block (four times the waves) shorten a lone
// generation (room20k: 0.05 ms of 0.93; Cornell: 0.01 of 0.24 ms), but under
// the render server those extra waves share the SIMDs with the other
// requests' gathers and the served median latency rises by about a tenth:
// full 64-lane waves are kept.
constexpr int kWalkLanes = 64;

// (block `blk` of the batch's blocks; no barrier inside)
__device__ __forceinline__ void walk_block(const DevScene& s, const DevLight& dl, const GenParams& p, const GenBuffers& b,
                           long long start, int nb, int blk, LdsStack stk)
{
    if ((int)threadIdx.x >= kWalkLanes) return;  // lanes past kWalkLanes idle
    int i = blk * kWalkLanes + threadIdx.x;
    if (i >= nb || b.state->walk_done) return;
    long long path = start + i + 1;
    b.w_count[i] = 0;
    if (path > (p.walk_schedule ? b.state->keller_n : (long long)p.max_paths) || (b.state->flags & 2)) return;
    Light64 L = light64(dl);
    int dim;
    d3 o, d;
    int ex = -1;
    bool skip_emit = false;
    if (L.kind == 0) {
        double u1 = halton(prime(0), path), u2 = halton(prime(1), path);
        double z = 1.0 - 2.0 * u1;
        double rr = sqrt(dmax(0.0, 1.0 - z * z));
        double phi = (2.0 * kPi) * u2;
        o = L.pos;
        d = mk(rr * cos(phi), rr * sin(phi), z);
        dim = 2;
    } else {
        double u1 = halton(prime(0), path), u2 = halton(prime(1), path);
        o = add(add(L.pos, scl(L.eu, u1)), scl(L.ev, u2));
        d = cos_dir(L.nl, halton(prime(2), path), halton(prime(3), path));
        dim = 4;
        skip_emit = true;
    }
    double flux[3] = {L.power[0], L.power[1], L.power[2]};
    int cnt = 0, discard_mask = 0;
    const double rb = s.rho_bar;
    for (int bnc = 1; bnc <= p.max_bounces; ++bnc) {
        if (p.walk_schedule && path > b.state->keller_t[bnc - 1]) break;
        double tb, u, v;
        int t = closest64(s, o, d, 0.0, ex, skip_emit, &tb, &u, &v, stk);
        if (t < 0) break;
        if (s.flags[t] & 1) break;
        d3 A = vA(s, t);
        d3 e1 = sub(vB(s, t), A), e2 = sub(vC(s, t), A);
        d3 nt = norm(cross(e1, e2));
        if (!(dot(d, nt) < 0.0)) break;
        for (int c = 0; c < 3; ++c) {
            flux[c] = flux[c] * (double)s.albedo[3 * t + c];
            if (p.walk_schedule && bnc >= 2) flux[c] = flux[c] / rb;
        }
        d3 y = add(add(A, scl(e1, u)), scl(e2, v));
        int n = b.level[t];
        double U = u * (double)n, V = v * (double)n;
        int a = (int)floor(U), bb = (int)floor(V);
        if (a < 0) a = 0;
        if (bb < 0) bb = 0;
        if (a > n - 1) a = n - 1;
        if (bb > n - 1) bb = n - 1;
        if (a + bb > n - 1) a = n - 1 - bb;
        int down = (a + bb <= n - 2) && ((U - (double)a) + (V - (double)bb) > 1.0);
        long long g = b.patch_off[t] + (long long)bb * (2 * n - bb) + 2 * a + down;
        if (!(b.pflags[g] & 1) || (p.walk_near == 1 && bnc >= 2)) {
            int slot = i * 3 + cnt;
            b.w_pos[3 * slot] = y.x; b.w_pos[3 * slot + 1] = y.y; b.w_pos[3 * slot + 2] = y.z;
            for (int c = 0; c < 3; ++c) b.w_flux[3 * slot + c] = flux[c];
            b.w_tri[slot] = t;
            b.w_bounce[slot] = bnc;
            cnt++;
        } else {
            discard_mask |= 1 << (bnc - 1);
            if (p.walk_near == 2) break;  // the near hit ends the path
        }
        if (bnc == p.max_bounces) break;
        double s1 = halton(prime(dim), path), s2 = halton(prime(dim + 1), path);
        dim += 2;
        o = y;
        d = cos_dir(nt, s1, s2);
        ex = t;
        skip_emit = false;
    }
    b.w_count[i] = cnt | (discard_mask << 8);
}

__global__ __launch_bounds__(kGenBlock) void k_walk(DevScene s, DevLight dl, GenParams p, GenBuffers b, long long start,
                                                    int nb)
{
    VPLG_LDS_STACK(stk);
    walk_block(s, dl, p, b, start, nb, blockIdx.x, stk);
}

// The near strata and the walk's first batch in one launch.  Both are
// latency-bound (few waves, long dependent FP64 traversals) and independent
// once k_strata_state has run (disjoint VPL ranges; the state they read is
// final), so they share the GPU instead of running one after the other:
// blocks [0, sb) place strata, the rest walk paths [start + 1, start + nb].
template <int S>
__global__ __launch_bounds__(kGenBlock) void k_strata_walk(DevScene s, DevLight dl, GenParams p, GenBuffers b, DevVpls v,
                                                           int sb, long long start, int nb)
{
    VPLG_LDS_STACK(stk);
    __shared__ double s_term[kGenBlock];
    if ((int)blockIdx.x < sb)
        strata_block<S>(s, dl, p, b, v, blockIdx.x, stk, s_term);
    else
        walk_block(s, dl, p, b, start, nb, blockIdx.x - sb, stk);
}

// One workgroup per batch: keep deposits in (path, bounce) order up to the
// far target, update the counts, and find the path that completes it.
constexpr int COLLECT_T = 1024;

__global__ __launch_bounds__(COLLECT_T) void k_walk_collect(GenParams p, GenBuffers b, DevVpls v, long long start,
                                                            int nb)
{
    __shared__ long long s_scan[COLLECT_T];
    __shared__ unsigned long long s_far[3], s_disc;
    __shared__ long long s_cut;
    GenState* st = b.state;
    if (st->walk_done) return;
    const long long have = st->n_far;
    // Keller's schedule keeps every deposit of its N paths (at most the target)
    const long long need = p.walk_schedule ? 0x7fffffffffffffffll : st->n_far_target;
    const int t = threadIdx.x;
    if (t < 3) s_far[t] = 0;
    if (t == 0) { s_disc = 0; s_cut = -1; }
    // contiguous chunk of paths per thread keeps (path, bounce) order
    const int chunk = (nb + COLLECT_T - 1) / COLLECT_T;
    const int i0 = t * chunk, i1 = min(nb, i0 + chunk);
    long long mine = 0;
    for (int i = i0; i < i1; ++i) mine += b.w_count[i] & 0xff;
    s_scan[t] = mine;
    __syncthreads();
    for (int off = 1; off < COLLECT_T; off <<= 1) {
        long long x = t >= off ? s_scan[t - off] : 0;
        __syncthreads();
        s_scan[t] += x;
        __syncthreads();
    }
    long long before = have + s_scan[t] - mine;
    const long long total = s_scan[COLLECT_T - 1];
    const long long base = st->k_eff;
    unsigned long long far_b[3] = {0, 0, 0}, disc = 0;
    for (int i = i0; i < i1 && before < need; ++i) {
        int cnt = b.w_count[i] & 0xff;
        int dmask = b.w_count[i] >> 8;
        long long keep = cnt;
        if (before + keep > need) keep = need - before;
        int last_bounce = 4;
        for (int j = 0; j < keep; ++j) {
            int slot = i * 3 + j;
            long long o = base + before + j;
            for (int c = 0; c < 3; ++c) {
                b.stage_pos[3 * o + c] = b.w_pos[3 * slot + c];
                b.stage_flux[3 * o + c] = b.w_flux[3 * slot + c];
            }
            v.tri[o] = b.w_tri[slot];
            b.vpl_path[o] = (int32_t)(start + i + 1);
            b.vpl_bounce[o] = b.w_bounce[slot];
            far_b[b.w_bounce[slot] - 1]++;
            last_bounce = b.w_bounce[slot];
        }
        // discards count up to the deposit that completes the target
        bool cut_here = before + cnt >= need;
        for (int bb = 1; bb <= 3; ++bb)
            if ((dmask >> (bb - 1)) & 1) disc += (!cut_here || bb < last_bounce) ? 1 : 0;
        if (cut_here) s_cut = start + i + 1;
        before += cnt;
    }
    for (int c = 0; c < 3; ++c)
        if (far_b[c]) atomicAdd(&s_far[c], far_b[c]);
    if (disc) atomicAdd(&s_disc, disc);
    __syncthreads();
    if (t == 0) {
        for (int c = 0; c < 3; ++c) st->far_b[c] += (long long)s_far[c];
        st->near_discarded += (long long)s_disc;
        if (s_cut >= 0) {
            st->n_paths = s_cut;
            st->n_far = need;
            st->walk_done = 1;
        } else {
            long long end = start + nb;
            st->n_far = have + total;
            const long long cap = p.walk_schedule ? st->keller_n : (long long)p.max_paths;
            if (end >= cap) {
                st->n_paths = cap;
                if (!p.walk_schedule) st->flags |= 1;
                st->walk_done = 1;
            } else {
                st->n_paths = end;
            }
        }
    }
}

// A zero far target needs no path at all.
// Divide far fluxes by the number of paths; I = flux / pi; write float VPLs.
__global__ void k_walk_finish(DevScene s, GenBuffers b, DevVpls v)
{
    long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    long long base = b.state->k_eff;
    long long nf = b.state->n_far;
    if (i == 0) *v.count = (int32_t)(base + nf);
    if (i >= nf) return;
    long long o = base + i;
    double np = (double)b.state->n_paths;
    float* outs[3] = {v.ir, v.ig, v.ib};
    for (int c = 0; c < 3; ++c) {
        double phi = b.stage_flux[3 * o + c] / np;
        outs[c][o] = (float)(phi / kPi);
    }
    v.px[o] = (float)b.stage_pos[3 * o]; v.py[o] = (float)b.stage_pos[3 * o + 1];
    v.pz[o] = (float)b.stage_pos[3 * o + 2];
    int t = v.tri[o];
    d3 A = vA(s, t);
    d3 nt = norm(cross(sub(vB(s, t), A), sub(vC(s, t), A)));
    v.nx[o] = (float)nt.x; v.ny[o] = (float)nt.y; v.nz[o] = (float)nt.z;
}

__device__ void state_init(const GenBuffers& b, long long n_patches)
{
    GenState* st = b.state;
    st->n_patches = n_patches;
    st->n_near = st->n_eligible = st->q_total = st->k_eff = st->n_far_target = st->n_far = st->n_paths = 0;
    st->far_b[0] = st->far_b[1] = st->far_b[2] = 0;
    st->flags = st->near_discarded = 0;
    st->keller_n = st->keller_t[0] = st->keller_t[1] = st->keller_t[2] = 0;
    st->walk_done = 0;
}

// The generation's state zeroed and the sort buffer filled with all-ones
// keys (one launch: both precede the classification).
__global__ void k_init_fill(GenBuffers b, long long n_patches, long long n2)
{
    long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i == 0) state_init(b, n_patches);
    if (i < n2) b.sortbuf[i] = ~0ull;
}

// ---------------------------------------------------------------------------
// int64 exclusive scan (three phases)
// ---------------------------------------------------------------------------
constexpr int SCAN_T = 256, SCAN_E = 8, SCAN_TILE = SCAN_T * SCAN_E;

__device__ long long block_excl_scan(long long v, long long* total)
{
    __shared__ long long s[SCAN_T];
    int t = threadIdx.x;
    s[t] = v;
    __syncthreads();
    for (int off = 1; off < SCAN_T; off <<= 1) {
        long long x = t >= off ? s[t - off] : 0;
        __syncthreads();
        s[t] += x;
        __syncthreads();
    }
    long long incl = s[t];
    *total = s[SCAN_T - 1];
    __syncthreads();
    return incl - v;
}

__global__ __launch_bounds__(SCAN_T) void k_scan_reduce(const long long* in, int n, long long* sums)
{
    long long base = (long long)blockIdx.x * SCAN_TILE;
    long long acc = 0;
    for (int e = 0; e < SCAN_E; ++e) {
        long long i = base + (long long)threadIdx.x * SCAN_E + e;
        if (i < n) acc += in[i];
    }
    long long total;
    block_excl_scan(acc, &total);
    if (threadIdx.x == 0) sums[blockIdx.x] = total;
}

__global__ __launch_bounds__(SCAN_T) void k_scan_sums(long long* sums, int nb)
{
    // single workgroup: exclusive scan of the per-tile sums, sums[nb] = total
    long long carry = 0;
    for (int base = 0; base < nb; base += SCAN_T) {
        int i = base + threadIdx.x;
        long long v = i < nb ? sums[i] : 0;
        long long total;
        long long ex = block_excl_scan(v, &total);
        if (i < nb) sums[i] = carry + ex;
        carry += total;
        __syncthreads();
    }
    if (threadIdx.x == 0) sums[nb] = carry;
}

__global__ __launch_bounds__(SCAN_T) void k_scan_apply(const long long* in, int n, const long long* sums,
                                                       long long* out)
{
    long long base = (long long)blockIdx.x * SCAN_TILE;
    long long v[SCAN_E];
    long long acc = 0;
    for (int e = 0; e < SCAN_E; ++e) {
        long long i = base + (long long)threadIdx.x * SCAN_E + e;
        v[e] = i < n ? in[i] : 0;
        acc += v[e];
    }
    long long total;
    long long ex = block_excl_scan(acc, &total) + sums[blockIdx.x];
    for (int e = 0; e < SCAN_E; ++e) {
        long long i = base + (long long)threadIdx.x * SCAN_E + e;
        if (i < n) out[i] = ex;
        ex += v[e];
    }
    if (blockIdx.x == gridDim.x - 1 && threadIdx.x == 0) out[n] = sums[gridDim.x];
}

// Small inputs: the whole exclusive scan in one workgroup, tile by tile with
// a running carry (integers: the same values as the three phases, in one
// launch instead of three).
constexpr int kScanSmallTiles = 16;

__global__ __launch_bounds__(SCAN_T) void k_scan_small(const long long* in, int n, long long* out)
{
    long long carry = 0;
    for (long long base = 0; base < n; base += SCAN_TILE) {
        long long v[SCAN_E];
        long long acc = 0;
        for (int e = 0; e < SCAN_E; ++e) {
            long long i = base + (long long)threadIdx.x * SCAN_E + e;
            v[e] = i < n ? in[i] : 0;
            acc += v[e];
        }
        long long total;
        long long ex = block_excl_scan(acc, &total) + carry;
        for (int e = 0; e < SCAN_E; ++e) {
            long long i = base + (long long)threadIdx.x * SCAN_E + e;
            if (i < n) out[i] = ex;
            ex += v[e];
        }
        carry += total;
    }
    if (threadIdx.x == 0) out[n] = carry;
}

inline unsigned nblocks(long long n, int b) { return (unsigned)((n + b - 1) / b); }

}  // namespace

int scan_tmp_needed(int n) { return (int)nblocks(n, SCAN_TILE) + 1; }

hipError_t launch_scan_i64(const long long* in, long long* out, int n, long long* tmp, int tmp_len, hipStream_t s)
{
    int nb = (int)nblocks(n, SCAN_TILE);
    if (nb < 1) nb = 1;
    if (tmp_len < nb + 1) return hipErrorInvalidValue;
    if (nb <= kScanSmallTiles) {
        hipLaunchKernelGGL(k_scan_small, dim3(1), dim3(SCAN_T), 0, s, in, n, out);
        return hipGetLastError();
    }
    hipLaunchKernelGGL(k_scan_reduce, dim3(nb), dim3(SCAN_T), 0, s, in, n, tmp);
    hipLaunchKernelGGL(k_scan_sums, dim3(1), dim3(SCAN_T), 0, s, tmp, nb);
    hipLaunchKernelGGL(k_scan_apply, dim3(nb), dim3(SCAN_T), 0, s, in, n, tmp, out);
    return hipGetLastError();
}

hipError_t launch_patch_levels(const DevScene& sc, double h, int32_t* level, long long* counts, hipStream_t s)
{
    hipLaunchKernelGGL(k_patch_levels, dim3(nblocks(sc.n_tris, GB)), dim3(GB), 0, s, sc, h, level, counts);
    return hipGetLastError();
}

// Enqueue the whole generation.  Device buffers in b are sized by the
// caller: sortbuf holds the next power of two >= max(n_patches, kLocal).
hipError_t launch_generate(const DevScene& sc, const DevLight& L, const CamBasis& cam, const GenParams& p,
                           const DevVpls& v, const GenBuffers& b, hipStream_t s)
{
    long long NP = b.n_patches;
    long long n2 = kLocal;
    while (n2 < NP) n2 <<= 1;
    hipLaunchKernelGGL(k_init_fill, dim3(nblocks(n2, GB)), dim3(GB), 0, s, b, NP, n2);
    if (NP > 0) hipLaunchKernelGGL(k_classify, dim3(nblocks(NP, GB)), dim3(GB), 0, s, sc, cam, L, p, b);
    // bitonic sort: LDS stages for j < kLocal, global passes above; the
    // network is launched for every patch, and its passes skip what lies past
    // the eligible keys' power of two (known on the device only)
    unsigned lb = (unsigned)(n2 / kLocal);
    hipLaunchKernelGGL(k_bitonic_local, dim3(lb), dim3(1024), 0, s, b.sortbuf, n2, 2ll, (long long)kLocal, 1ll,
                       (const GenState*)b.state);
    for (long long k = 2ll * kLocal; k <= n2; k <<= 1) {
        for (long long j = k >> 1; j >= kLocal; j >>= 1)
            hipLaunchKernelGGL(k_bitonic_global, dim3(nblocks(n2, GB)), dim3(GB), 0, s, b.sortbuf, n2, j, k,
                               (const GenState*)b.state);
        hipLaunchKernelGGL(k_bitonic_local, dim3(lb), dim3(1024), 0, s, b.sortbuf, n2, k, k, (long long)(kLocal / 2),
                           (const GenState*)b.state);
    }
    // fixed-point areas -> inclusive prefix F
    if (NP > 0) {
        hipLaunchKernelGGL(k_sorted_areas, dim3(nblocks(NP, GB)), dim3(GB), 0, s, sc, p, b, b.q);
        hipError_t e = launch_scan_i64(b.q, b.scan_out, (int)NP, b.scan_tmp, b.scan_tmp_len, s);
        if (e != hipSuccess) return e;
    }
    GenBuffers bb = b;
    bb.F = b.scan_out + 1;
    bb.patch_g = reinterpret_cast<double*>(b.sortbuf);
    if (p.brightness && p.k_near > 0 && NP > 0)
    {
        // quad light: one lane per light sample (16 per patch)
        if (L.kind == 1)
            hipLaunchKernelGGL(k_patch_light<16>, dim3(nblocks(NP * 16, kGenBlock)), dim3(kGenBlock), 0, s, sc, L, p, bb);
        else
            hipLaunchKernelGGL(k_patch_light<1>, dim3(nblocks(NP, kGenBlock)), dim3(kGenBlock), 0, s, sc, L, p, bb);
    }
    hipLaunchKernelGGL(k_strata_state, dim3(1), dim3(1), 0, s, p, bb, sc.rho_bar);
    // the walk: batches until the far target is met or max_paths is reached
    // (batches after that exit at once; k_strata_state marks a zero target
    // done)
    long long start = 0;
    // the walk is latency-bound (one serial path per thread): every batch
    // takes the whole capacity; deposits are kept in path order, so the batch
    // sizes never change the result.  The first batch runs in one launch with
    // the near strata (quad light and eq. (2) at the VPL's point: one lane
    // per light sample).
    int nb = b.batch;
    const bool quad = L.kind == 1 && !p.brightness;
    const int sb = p.k_near > 0 ? (int)nblocks((long long)p.k_near * (quad ? 16 : 1), kGenBlock) : 0;
    const unsigned fused = (unsigned)(sb + nblocks(nb, kWalkLanes));
    if (quad)
        hipLaunchKernelGGL(k_strata_walk<16>, dim3(fused), dim3(kGenBlock), 0, s, sc, L, p, bb, v, sb, start, nb);
    else
        hipLaunchKernelGGL(k_strata_walk<1>, dim3(fused), dim3(kGenBlock), 0, s, sc, L, p, bb, v, sb, start, nb);
    hipLaunchKernelGGL(k_walk_collect, dim3(1), dim3(COLLECT_T), 0, s, p, bb, v, start, nb);
    start += nb;
    while (start < p.max_paths) {
        hipLaunchKernelGGL(k_walk, dim3(nblocks(nb, kWalkLanes)), dim3(kGenBlock), 0, s, sc, L, p, bb, start, nb);
        hipLaunchKernelGGL(k_walk_collect, dim3(1), dim3(COLLECT_T), 0, s, p, bb, v, start, nb);
        start += nb;
        nb = nb * 2 <= b.batch ? nb * 2 : b.batch;
    }
    hipLaunchKernelGGL(k_walk_finish, dim3(nblocks(v.capacity > 0 ? v.capacity : 1, GB)), dim3(GB), 0, s, sc, bb, v);
    return hipGetLastError();
}

}  // namespace vplg
