// FP32 kernels of the VPL gather (eq. (1) without the direct term), its
// visibility dump, and the primary-ray G-buffer.
//
// Every shadow ray is the segment x + s (y - x), s in (t_eps, 1 - t_eps),
// tested against the BVH with both host triangles excluded; occlusion is
// two-sided and emitters occlude.
//
// Each segment's range is first clipped at both ends by the free radii of its
// end points (the distance within which nothing but the point's own surface
// plane lies; see free_radius): the parts of the segment next to its end
// surfaces, where a walk spends many of its node steps, need no test.
//
// Shadow rays are traced as wave64 packets: a wave owns an 8 x 8 pixel tile
// and all 64 rays run to the same VPL, so they are coherent.  The wave walks
// the BVH together with uniform control flow: node and triangle records are
// wave-uniform loads (scalar unit, SGPRs), each lane tests its own ray, and
// ballots decide which children the packet enters.  The traversal stack is
// wave-uniform and lives in one VGPR across the lanes (entry i in lane i:
// push by lane select, pop by v_readlane), so it costs no LDS at all.
//
// A resident grid of workgroups claims work items from a device counter:
// whole tiles, and at the end of a long view quarter tiles (one round group of
// VPLs each) whose sums a second kernel adds up.  A pixel's sum is fixed as
// chunk, round-group, wave and group order, so its value never depends on how
// the items were dealt out.
#include <algorithm>
#include <mutex>

#include "vplg_impl.h"

namespace vplg {

namespace {

constexpr int BLOCK = 256;              // 4 wave64 per workgroup (G-buffer, dump)
constexpr int kGatherMaxWaves = 16;     // waves per gather workgroup (VPL slices of one tile)
constexpr int kGatherMaxThreads = 64 * kGatherMaxWaves;
constexpr int kChunk = 16;              // VPLs per first-level partial sum of a wave
constexpr int kGroups = 4;              // round groups of a tile (the split granularity of the tail)
constexpr int kSplitRounds = 2;         // split blocks per workgroup of the launch
constexpr float kInvPi = 0.318309886183790671538f;
// Free radius of a surface point (see free_radius): triangles whose vertices
// all lie within kFreeCoplanar x the scene diagonal of the point's plane count
// as lying in it, and the radius is shortened by kFreeMargin x the largest
// coordinate magnitude (plus 2^-12 of itself) against its FP32 rounding.
constexpr float kFreeCoplanar = 4e-8f;
constexpr float kFreeMargin = 2e-6f;
// The radius is sought no farther than a cap x the scene diagonal (the walk
// prunes every box beyond it): a receiver's walk, once per tile inside the
// gather, stops at kFreeCapTile (the clipping gains little more from larger
// radii there), a VPL's, one wave per VPL before the gather, at kFreeCapVpl.
constexpr float kFreeCapTile = 0.05f;
constexpr float kFreeCapVpl = 0.2f;

// Work memory of the allocation-free gather: the tile counter in the first
// 256 bytes, then the round-group sums of at most kScratchSplitTiles split
// tiles (6,291,712 bytes in all).  A file-scope device array: every device
// the library runs on holds its own copy until the process ends, and every
// allocation-free gather on that device shares it.
constexpr int kScratchSplitTiles = 2048;
constexpr size_t kScratchBytes = 256 + (size_t)kScratchSplitTiles * kGroups * 3 * 64 * sizeof(float);
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

__device__ __forceinline__ float rcpf(float x) { return __builtin_amdgcn_rcpf(x); }

// One 64-byte node or triangle record, fetched by a single load (a scalar
// s_load_dwordx16 when the index is wave-uniform).  Scenes hold at most 2^25
// triangles, so a record's byte offset fits in 32 bits.  Scene and VPL
// records are read through the constant address space: no kernel here writes
// them, and saying so lets the compiler use scalar loads even where the
// kernel's own stores (a persistent loop's outputs) precede the load.
typedef float Rec16 __attribute__((ext_vector_type(16)));
#define VPLG_CONST __attribute__((address_space(4)))

struct Rec {
    float4 q0, q1, q2, q3;
};

typedef float F4v __attribute__((ext_vector_type(4)));

__device__ __forceinline__ float4 load_c4(const float4* __restrict__ p, int i)
{
    const F4v v = ((const VPLG_CONST F4v*)p)[i];
    return make_float4(v.x, v.y, v.z, v.w);
}

__device__ __forceinline__ Rec load_rec(const float4* __restrict__ base, int idx)
{
    const Rec16 v = *(const VPLG_CONST Rec16*)((const VPLG_CONST char*)base + (size_t)((unsigned)idx << 6));
    Rec r;
    r.q0 = make_float4(v.s0, v.s1, v.s2, v.s3);
    r.q1 = make_float4(v.s4, v.s5, v.s6, v.s7);
    r.q2 = make_float4(v.s8, v.s9, v.sa, v.sb);
    r.q3 = make_float4(v.sc, v.sd, v.se, v.sf);
    return r;
}

__device__ __forceinline__ float safe_inv(float d)
{
    // A zero direction component would turn the slab test into 0 * inf; the
    // reciprocal clamped to +-1e30 keeps the slab unbounded on that axis.
    return __builtin_amdgcn_fmed3f(rcpf(d), -1e30f, 1e30f);
}

// Counters of the instrumented gather.  Per lane: shadow rays cast, BVH node
// visits of the ray's own traversal (nodes its segment entered), triangle
// tests of the ray's own traversal, node steps the lane rode along unblocked
// (its own and the packet's), and rays found blocked.  Per wave: packets
// traced, packet node steps, active lanes at packet start, packet triangle
// steps, steps entering both children, steps entering neither (a pop), and
// packets with every ray blocked or none.
constexpr int kCounters = 14;
struct Counters {
    unsigned long long rays = 0, nodes = 0, tris = 0;
    unsigned long long packets = 0, psteps = 0, plane = 0, ptris = 0;
    unsigned long long rides = 0, both = 0, pops = 0, pk_blocked = 0, pk_clear = 0, blocked = 0;
};

// Per-ray set-up of the watertight ray/triangle test (Woop, Benthin and
// Wald 2013): the dominant direction axis kz, the two others kx, ky in cyclic
// order, and the shear/scale taking the ray to the +z axis through the
// origin.  The test is two-sided, so the kx/ky swap the paper uses to keep
// the winding for d[kz] < 0 is left out: it would only negate all three edge
// functions, the determinant and T exactly.
struct WtRay {
    float ox, oy, oz;
    float sx, sy, sz;
    float q;  // |d|^2 / d[kz]^2: scales the parallel-ray cut to the determinant
    int kx, ky, kz;
    // pre: the records come from the scene's plane for this ray's kz (their
    // vertices already permuted), and o[kx], o[ky], o[kz] are given
    bool pre;
    float okx, oky, okz;
};

__device__ __forceinline__ float sel3(float x, float y, float z, int k) { return k == 0 ? x : (k == 1 ? y : z); }

__device__ __forceinline__ WtRay wt_ray(float ox, float oy, float oz, float dx, float dy, float dz)
{
    WtRay r;
    r.ox = ox; r.oy = oy; r.oz = oz;
    const float ax = fabsf(dx), ay = fabsf(dy), az = fabsf(dz);
    r.kz = ax > ay ? (ax > az ? 0 : 2) : (ay > az ? 1 : 2);
    r.kx = r.kz == 2 ? 0 : r.kz + 1;
    r.ky = r.kx == 2 ? 0 : r.kx + 1;
    const float dkz = sel3(dx, dy, dz, r.kz);
    r.sz = rcpf(dkz);
    r.sx = sel3(dx, dy, dz, r.kx) * r.sz;
    r.sy = sel3(dx, dy, dz, r.ky) * r.sz;
    r.q = fmaf(r.sy, r.sy, fmaf(r.sx, r.sx, 1.0f));
    r.pre = false;
    r.okx = r.oky = r.okz = 0.f;
    return r;
}

// Watertight test of one leaf-ordered triangle record (two-sided).  The ray
// crosses the closed triangle iff the edge functions U, V, W are not of mixed
// sign and their sum (the determinant) is non-zero; the hit parameter is
// T / det.  The determinant equals d . n / d[kz] (n = (B - A) x (C - A)), so
// the parallel-ray cut |d . n| > kParallelTau |d| |n| reads
// det^2 > cut q with the stored cut = (kParallelTau |n|)^2 (infinite for a
// degenerate triangle).  The file is built without floating-point
// contraction, so every product below is rounded on its own unless written
// as fmaf.
struct TriEval {
    float U, V, W, det, t, inv;
    float akz, bkz, ckz;  // vertex depths along the dominant axis, relative to the origin
    bool steep;
    int id;
};

// First half of the test: the edge functions U, V, W (their signs decide
// whether the ray's line crosses the triangle).
__device__ __forceinline__ TriEval tri_edges(const Rec& rec, const WtRay& r)
{
    const float4 q0 = rec.q0, q1 = rec.q1, q2 = rec.q2;
    TriEval e;
    e.id = __float_as_int(q0.w);
    // vertices relative to the ray origin, permuted (a[kx], a[ky], a[kz]) ...
    float akx, aky, akz, bkx, bky, bkz, ckx, cky, ckz;
    if (r.pre) {
        // ... by the record's plane already
        akx = q0.x - r.okx, aky = q0.y - r.oky, akz = q0.z - r.okz;
        bkx = q1.x - r.okx, bky = q1.y - r.oky, bkz = q1.z - r.okz;
        ckx = q2.x - r.okx, cky = q2.y - r.oky, ckz = q2.z - r.okz;
    } else {
        // ... or per lane (the same differences, selected afterwards)
        const float ax = q0.x - r.ox, ay = q0.y - r.oy, az = q0.z - r.oz;
        const float bx = q1.x - r.ox, by = q1.y - r.oy, bz = q1.z - r.oz;
        const float cx = q2.x - r.ox, cy = q2.y - r.oy, cz = q2.z - r.oz;
        akx = sel3(ax, ay, az, r.kx), aky = sel3(ax, ay, az, r.ky), akz = sel3(ax, ay, az, r.kz);
        bkx = sel3(bx, by, bz, r.kx), bky = sel3(bx, by, bz, r.ky), bkz = sel3(bx, by, bz, r.kz);
        ckx = sel3(cx, cy, cz, r.kx), cky = sel3(cx, cy, cz, r.ky), ckz = sel3(cx, cy, cz, r.kz);
    }
    // ... and sheared into ray space
    const float Ax = fmaf(-r.sx, akz, akx), Ay = fmaf(-r.sy, akz, aky);
    const float Bx = fmaf(-r.sx, bkz, bkx), By = fmaf(-r.sy, bkz, bky);
    const float Cx = fmaf(-r.sx, ckz, ckx), Cy = fmaf(-r.sy, ckz, cky);
    // edge functions: products rounded separately, so the two triangles of a
    // shared edge compute exact negatives of each other
    float U = Cx * By - Cy * Bx;
    float V = Ax * Cy - Ay * Cx;
    float W = Bx * Ay - By * Ax;
    if (fminf(fminf(fabsf(U), fabsf(V)), fabsf(W)) == 0.f) {
        // exact sign on an edge: float products are exact in double
        U = (float)((double)Cx * (double)By - (double)Cy * (double)Bx);
        V = (float)((double)Ax * (double)Cy - (double)Ay * (double)Cx);
        W = (float)((double)Bx * (double)Ay - (double)By * (double)Ax);
    }
    e.U = U;
    e.V = V;
    e.W = W;
    e.akz = akz;
    e.bkz = bkz;
    e.ckz = ckz;
    return e;
}

// Second half: determinant, hit parameter and the parallel-ray cut.
__device__ __forceinline__ void tri_finish(TriEval& e, const Rec& rec, const WtRay& r)
{
    e.det = e.U + e.V + e.W;
    // t = T / det with T = sz (U a_kz + V b_kz + W c_kz)
    const float T = fmaf(e.W, e.ckz, fmaf(e.V, e.bkz, e.U * e.akz));
    e.inv = rcpf(e.det);
    e.t = T * (r.sz * e.inv);
    e.steep = e.det * e.det > rec.q1.w * r.q;
}

__device__ __forceinline__ TriEval tri_eval(const Rec& rec, const WtRay& r)
{
    TriEval e = tri_edges(rec, r);
    tri_finish(e, rec, r);
    return e;
}

// Per-lane hit test for the closest-hit walk: parameter in (tlo, thi).
__device__ __forceinline__ bool tri_hit32(const Rec& rec, const WtRay& r, float tlo, float thi, float* tout,
                                          float* uout, float* vout, int* idout)
{
    const TriEval e = tri_eval(rec, r);
    const bool mixed = fminf(fminf(e.U, e.V), e.W) < 0.f && fmaxf(fmaxf(e.U, e.V), e.W) > 0.f;
    *tout = e.t;
    *uout = e.V * e.inv;
    *vout = e.W * e.inv;
    *idout = e.id;
    return !mixed && e.det != 0.f && e.steep && e.t > tlo && e.t < thi;
}

struct SlabRay {
    float ix, iy, iz, ox, oy, oz;  // inverse direction and origin * inverse
};

// Slab test of both child boxes of a node for a ray with parameter range
// (tlo, thi) and any direction signs (the G-buffer's primary rays).
__device__ __forceinline__ void child_boxes(const float4& n0, const float4& n1, const float4& n2, const SlabRay& r,
                                            float tlo, float thi, float* lo0, float* hi0, float* lo1, float* hi1)
{
    const float a0 = fmaf(n0.x, r.ix, -r.ox), a1 = fmaf(n0.y, r.ix, -r.ox);
    const float b0 = fmaf(n0.z, r.iy, -r.oy), b1 = fmaf(n0.w, r.iy, -r.oy);
    const float c0 = fmaf(n2.x, r.iz, -r.oz), c1 = fmaf(n2.y, r.iz, -r.oz);
    *lo0 = fmaxf(fmaxf(fminf(a0, a1), fminf(b0, b1)), fmaxf(fminf(c0, c1), tlo));
    *hi0 = fminf(fminf(fmaxf(a0, a1), fmaxf(b0, b1)), fminf(fmaxf(c0, c1), thi));
    const float d0 = fmaf(n1.x, r.ix, -r.ox), d1 = fmaf(n1.y, r.ix, -r.ox);
    const float e0 = fmaf(n1.z, r.iy, -r.oy), e1 = fmaf(n1.w, r.iy, -r.oy);
    const float f0 = fmaf(n2.z, r.iz, -r.oz), f1 = fmaf(n2.w, r.iz, -r.oz);
    *lo1 = fmaxf(fmaxf(fminf(d0, d1), fminf(e0, e1)), fmaxf(fminf(f0, f1), tlo));
    *hi1 = fminf(fminf(fmaxf(d0, d1), fmaxf(e0, e1)), fminf(fmaxf(f0, f1), thi));
}

// Slab test of both child boxes of a node for a segment whose SlabRay is
// rescaled to its parameter range: plane distances are u = (s - tlo) /
// (thi - tlo), so the range is u in [0, 1].  Every distance is clamped to
// [0, 1] (a free output modifier of the FMA), which folds in the range
// limits: a child passes iff lo < hi, i.e. the segment crosses the box over
// an interval of positive length.  That is the exact-range test except for
// zero-length contacts (lo == hi), and those cannot lead to a triangle:
// boxes are padded outward by more than the FP32 error of the plane
// distances, so a segment through a point of a triangle crosses the box of
// every node holding it over an interval longer than that error.  No plane
// distance is NaN (safe_inv keeps the inverse direction finite).
__device__ __forceinline__ float clamp01(float x) { return __builtin_amdgcn_fmed3f(x, 0.f, 1.f); }

template <int OCT>
__device__ __forceinline__ void seg_boxes(const float4& n0, const float4& n1, const float4& n2, const SlabRay& r,
                                          float* lo0, float* hi0, float* lo1, float* hi1)
{
    if constexpr (OCT < 8) {
        constexpr bool nx = OCT & 1, ny = OCT & 2, nz = OCT & 4;
        const float a0 = clamp01(fmaf(nx ? n0.y : n0.x, r.ix, -r.ox)), a1 = clamp01(fmaf(nx ? n0.x : n0.y, r.ix, -r.ox));
        const float b0 = clamp01(fmaf(ny ? n0.w : n0.z, r.iy, -r.oy)), b1 = clamp01(fmaf(ny ? n0.z : n0.w, r.iy, -r.oy));
        const float c0 = clamp01(fmaf(nz ? n2.y : n2.x, r.iz, -r.oz)), c1 = clamp01(fmaf(nz ? n2.x : n2.y, r.iz, -r.oz));
        *lo0 = fmaxf(fmaxf(a0, b0), c0);
        *hi0 = fminf(fminf(a1, b1), c1);
        const float d0 = clamp01(fmaf(nx ? n1.y : n1.x, r.ix, -r.ox)), d1 = clamp01(fmaf(nx ? n1.x : n1.y, r.ix, -r.ox));
        const float e0 = clamp01(fmaf(ny ? n1.w : n1.z, r.iy, -r.oy)), e1 = clamp01(fmaf(ny ? n1.z : n1.w, r.iy, -r.oy));
        const float f0 = clamp01(fmaf(nz ? n2.w : n2.z, r.iz, -r.oz)), f1 = clamp01(fmaf(nz ? n2.z : n2.w, r.iz, -r.oz));
        *lo1 = fmaxf(fmaxf(d0, e0), f0);
        *hi1 = fminf(fminf(d1, e1), f1);
    } else {
        const float a0 = clamp01(fmaf(n0.x, r.ix, -r.ox)), a1 = clamp01(fmaf(n0.y, r.ix, -r.ox));
        const float b0 = clamp01(fmaf(n0.z, r.iy, -r.oy)), b1 = clamp01(fmaf(n0.w, r.iy, -r.oy));
        const float c0 = clamp01(fmaf(n2.x, r.iz, -r.oz)), c1 = clamp01(fmaf(n2.y, r.iz, -r.oz));
        *lo0 = fmaxf(fmaxf(fminf(a0, a1), fminf(b0, b1)), fminf(c0, c1));
        *hi0 = fminf(fminf(fmaxf(a0, a1), fmaxf(b0, b1)), fmaxf(c0, c1));
        const float d0 = clamp01(fmaf(n1.x, r.ix, -r.ox)), d1 = clamp01(fmaf(n1.y, r.ix, -r.ox));
        const float e0 = clamp01(fmaf(n1.z, r.iy, -r.oy)), e1 = clamp01(fmaf(n1.w, r.iy, -r.oy));
        const float f0 = clamp01(fmaf(n2.z, r.iz, -r.oz)), f1 = clamp01(fmaf(n2.w, r.iz, -r.oz));
        *lo1 = fmaxf(fmaxf(fminf(d0, d1), fminf(e0, e1)), fminf(f0, f1));
        *hi1 = fminf(fminf(fmaxf(d0, d1), fmaxf(e0, e1)), fmaxf(f0, f1));
    }
}

__device__ __forceinline__ unsigned long long ballot(bool p) { return __builtin_amdgcn_ballot_w64(p); }

__device__ __forceinline__ bool lane_bit(unsigned long long m, int lane) { return (m >> lane) & 1ull; }

// Any-hit test of the packet lanes in `enter` (a subset of `alive`) against
// the triangles [first, first + count) of one leaf.  Returns `alive` with
// the blocked lanes cleared; stops early once every entering lane is blocked.
template <bool COUNT>
__device__ __forceinline__ unsigned long long leaf_any_hit(const float4* __restrict__ tris, int first, int count,
                                                           const WtRay& wr, float tlo, float thi, int ex0, int ex1,
                                                           unsigned long long enter, unsigned long long alive, int lane,
                                                           Counters& cnt)
{
    for (int i = first; i < first + count; ++i) {
        if (COUNT && lane_bit(enter & alive, lane)) cnt.tris++;
        if (COUNT && lane == 0) cnt.ptris++;
        const Rec rec = load_rec(tris, i);
        if (__float_as_int(rec.q0.w) == ex1) continue;  // the VPL's own triangle
        TriEval e = tri_edges(rec, wr);
        // lanes whose line crosses the triangle; the masks of the single
        // conditions combine on the scalar unit
        const unsigned long long inside = (ballot(fminf(fminf(e.U, e.V), e.W) >= 0.f) |
                                           ballot(fmaxf(fmaxf(e.U, e.V), e.W) <= 0.f)) & enter & alive;
        // most tests end here: no entering lane's line crosses the triangle
        if (inside == 0) continue;
        tri_finish(e, rec, wr);
        // steep implies det != 0 (det^2 > cut q > 0)
        const unsigned long long blocked = inside & ballot(e.steep) & ballot(e.t > tlo) & ballot(e.t < thi) &
                                           ballot(e.id != ex0);
        alive &= ~blocked;
        if ((alive & enter) == 0) break;
    }
    return alive;
}

// Order-preserving integer key of a float (as the node records store their
// split positions): integer comparison of keys is float comparison.
__device__ __forceinline__ int order_key(float f)
{
    const int b = __float_as_int(f);
    return b ^ ((b >> 31) & 0x7fffffff);
}

// BVH walk of one packet (see packet_visible) with slab-test variant OCT.
// Where the packet enters both children, it goes first to the one on the
// side of the split holding the midpoint (keys mk) of its lead segment:
// shadow rays are mostly blocked between their ends, away from the surfaces
// they start and end on, so the middle first finds a blocker sooner (on the
// 202k-triangle room a blocked packet took 49 node steps near side first
// and takes about 32 this way).
template <bool COUNT, int OCT>
__device__ __forceinline__ bool traverse(const float4* __restrict__ nodes, const float4* __restrict__ tris,
                                         const SlabRay& r, const WtRay& wr, bool act, float tlo, float thi, int ex0,
                                         int ex1, int mkx, int mky, int mkz, int lane, Counters& cnt)
{
    unsigned long long alive = ballot(act);
    int slot = 0;
    int sp = 0;
    int node = 0;
    // instrumented only: the lanes whose own segment entered `node` (the
    // parent's slab test of that child passed for them), kept on a second
    // stack beside the node index
    unsigned long long entered = alive;
    unsigned int slot_lo = 0, slot_hi = 0;
    while (true) {
        const Rec nd = load_rec(nodes, node);
        const float4 n0 = nd.q0, n1 = nd.q1, n2 = nd.q2, n3f = nd.q3;
        const int c0 = __float_as_int(n3f.x), c1 = __float_as_int(n3f.y);
        const int kk = __float_as_int(n3f.z), split = __float_as_int(n3f.w);
        if (COUNT) {
            if (lane_bit(entered & alive, lane)) cnt.nodes++;
            if (lane_bit(alive, lane)) cnt.rides++;
            if (lane == 0) cnt.psteps++;
        }
        float lo0, hi0, lo1, hi1;
        seg_boxes<OCT>(n0, n1, n2, r, &lo0, &hi0, &lo1, &hi1);
        unsigned long long b0 = ballot(lo0 < hi0) & alive;
        unsigned long long b1 = ballot(lo1 < hi1) & alive;
        if (kk != 0) {
            // a leaf child is tested at once and never entered
            const int k0 = kk & 0xffff, k1 = kk >> 16;
            if (k0 > 0) {
                if (b0) alive = leaf_any_hit<COUNT>(tris, c0, k0, wr, tlo, thi, ex0, ex1, b0, alive, lane, cnt);
                b0 = 0;
            }
            if (k1 > 0) {
                if (b1 & alive) alive = leaf_any_hit<COUNT>(tris, c1, k1, wr, tlo, thi, ex0, ex1, b1, alive, lane, cnt);
                b1 = 0;
            }
            if (alive == 0) break;
            b0 &= alive;
            b1 &= alive;
        }
        if (b0) {
            if (b1) {
                // both: the child on the midpoint's side of the split first,
                // the other pushed (uniform values: scalar compares)
                const int axis = split & 3;
                const int mk = axis == 0 ? mkx : (axis == 1 ? mky : mkz);
                const bool first1 = mk > (split & ~3);
                slot = lane == sp ? (first1 ? c0 : c1) : slot;
                if (COUNT) {
                    const unsigned long long later = first1 ? b0 : b1;
                    slot_lo = lane == sp ? (unsigned int)later : slot_lo;
                    slot_hi = lane == sp ? (unsigned int)(later >> 32) : slot_hi;
                    entered = first1 ? b1 : b0;
                    if (lane == 0) cnt.both++;
                }
                ++sp;
                node = first1 ? c1 : c0;
            } else {
                node = c0;
                if (COUNT) entered = b0;
            }
        } else if (b1) {
            node = c1;
            if (COUNT) entered = b1;
        } else {
            if (COUNT && lane == 0) cnt.pops++;
            if (sp == 0) break;
            --sp;
            node = __builtin_amdgcn_readlane(slot, sp);
            if (COUNT)
                entered = (unsigned long long)(unsigned int)__builtin_amdgcn_readlane((int)slot_lo, sp) |
                          ((unsigned long long)(unsigned int)__builtin_amdgcn_readlane((int)slot_hi, sp) << 32);
        }
    }
    return lane_bit(alive, lane);
}

// Squared distance from p to a box (0 inside it).
__device__ __forceinline__ float box_dist2(float px, float py, float pz, float lx, float hx, float ly, float hy, float lz,
                                           float hz)
{
    const float ex = fmaxf(fmaxf(lx - px, px - hx), 0.f);
    const float ey = fmaxf(fmaxf(ly - py, py - hy), 0.f);
    const float ez = fmaxf(fmaxf(lz - pz, pz - hz), 0.f);
    return fmaf(ez, ez, fmaf(ey, ey, ex * ex));
}

// Squared distance from p to the segment a + t e, t in [0, 1], with w = p - a.
__device__ __forceinline__ float seg_dist2(float wx, float wy, float wz, float ex, float ey, float ez)
{
    const float ee = fmaf(ez, ez, fmaf(ey, ey, ex * ex));
    const float we = fmaf(wz, ez, fmaf(wy, ey, wx * ex));
    const float t = ee > 0.f ? fminf(fmaxf(we / ee, 0.f), 1.f) : 0.f;
    const float vx = fmaf(-t, ex, wx), vy = fmaf(-t, ey, wy), vz = fmaf(-t, ez, wz);
    return fmaf(vz, vz, fmaf(vy, vy, vx * vx));
}

// Squared distance from p to triangle ABC: to its plane where p projects
// inside it, else to the nearest edge.  Near an edge the two agree, so an
// inside test that FP32 rounding gets wrong there costs next to nothing.
__device__ __forceinline__ float tri_dist2(float px, float py, float pz, const Rec& rec)
{
    const float ax = rec.q0.x, ay = rec.q0.y, az = rec.q0.z;
    const float e0x = rec.q1.x - ax, e0y = rec.q1.y - ay, e0z = rec.q1.z - az;  // B - A
    const float e1x = rec.q2.x - ax, e1y = rec.q2.y - ay, e1z = rec.q2.z - az;  // C - A
    const float e2x = rec.q2.x - rec.q1.x, e2y = rec.q2.y - rec.q1.y, e2z = rec.q2.z - rec.q1.z;  // C - B
    const float w0x = px - ax, w0y = py - ay, w0z = pz - az;
    const float w1x = px - rec.q1.x, w1y = py - rec.q1.y, w1z = pz - rec.q1.z;
    const float w2x = px - rec.q2.x, w2y = py - rec.q2.y, w2z = pz - rec.q2.z;
    const float nx = e0y * e1z - e0z * e1y, ny = e0z * e1x - e0x * e1z, nz = e0x * e1y - e0y * e1x;
    const float nn = fmaf(nz, nz, fmaf(ny, ny, nx * nx));
    // p's projection is inside iff it is on the inner side of all three edges
    auto side = [&](float ex, float ey, float ez, float wx, float wy, float wz) {
        const float cx = ey * wz - ez * wy, cy = ez * wx - ex * wz, cz = ex * wy - ey * wx;
        return fmaf(nz, cz, fmaf(ny, cy, nx * cx));
    };
    const bool inside = nn > 0.f && side(e0x, e0y, e0z, w0x, w0y, w0z) >= 0.f &&
                        side(e2x, e2y, e2z, w1x, w1y, w1z) >= 0.f && side(-e1x, -e1y, -e1z, w2x, w2y, w2z) >= 0.f;
    const float h = fmaf(nz, w0z, fmaf(ny, w0y, nx * w0x));
    const float dp = inside ? h * h / nn : __builtin_inff();
    const float de = fminf(fminf(seg_dist2(w0x, w0y, w0z, e0x, e0y, e0z), seg_dist2(w1x, w1y, w1z, e2x, e2y, e2z)),
                           seg_dist2(w0x, w0y, w0z, e1x, e1y, e1z));
    return fminf(dp, de);
}

// Whether triangle `rec`'s bounding box is nearer to p than best2 (squared):
// only then can the triangle lower p's nearest distance.
__device__ __forceinline__ bool free_tri_near(float px, float py, float pz, const Rec& rec, float best2)
{
    const float lx = fminf(fminf(rec.q0.x, rec.q1.x), rec.q2.x), hx = fmaxf(fmaxf(rec.q0.x, rec.q1.x), rec.q2.x);
    const float ly = fminf(fminf(rec.q0.y, rec.q1.y), rec.q2.y), hy = fmaxf(fmaxf(rec.q0.y, rec.q1.y), rec.q2.y);
    const float lz = fminf(fminf(rec.q0.z, rec.q1.z), rec.q2.z), hz = fmaxf(fmaxf(rec.q0.z, rec.q1.z), rec.q2.z);
    return box_dist2(px, py, pz, lx, hx, ly, hy, lz, hz) <= best2;
}

// Whether a box lies within `tol` of the plane through p with unit normal n
// (its farthest corner from the plane is no farther): every triangle in it
// then lies in p's plane and cannot lower p's free radius.
__device__ __forceinline__ bool box_in_plane(float px, float py, float pz, float nx, float ny, float nz, float lx,
                                             float hx, float ly, float hy, float lz, float hz, float tol)
{
    const float c = fmaf(nz, 0.5f * (lz + hz) - pz, fmaf(ny, 0.5f * (ly + hy) - py, nx * (0.5f * (lx + hx) - px)));
    const float e = fmaf(fabsf(nz), 0.5f * (hz - lz), fmaf(fabsf(ny), 0.5f * (hy - ly), fabsf(nx) * (0.5f * (hx - lx))));
    return fabsf(c) + e <= tol;
}

// Coplanarity tolerance, safety margin and squared cap of the free radius in
// a scene.
__device__ __forceinline__ void free_bounds(const DevScene& sc, float cap, float* tol, float* margin, float* cap2)
{
    const float dx = sc.hi[0] - sc.lo[0], dy = sc.hi[1] - sc.lo[1], dz = sc.hi[2] - sc.lo[2];
    const float diag = sqrtf(fmaf(dz, dz, fmaf(dy, dy, dx * dx)));
    *tol = kFreeCoplanar * diag;
    *cap2 = (cap * diag) * (cap * diag);
    const float big = fmaxf(fmaxf(fmaxf(fabsf(sc.lo[0]), fabsf(sc.hi[0])), fmaxf(fabsf(sc.lo[1]), fabsf(sc.hi[1]))),
                            fmaxf(fabsf(sc.lo[2]), fabsf(sc.hi[2])));
    *margin = kFreeMargin * big;
}

// The free radius from the squared nearest distance: shortened by 2^-12 of
// itself and by the margin, never below 0.
__device__ __forceinline__ float free_safe(float best2, float margin)
{
    const float r = sqrtf(best2);
    return fmaxf(0.f, fmaf(r, -1.0f / 4096.0f, r) - margin);
}

// Free radius of the surface points of a wave's lanes: a lower bound on the
// distance from p to every triangle but p's own (ex) and those lying in p's
// surface plane (unit normal n; all three vertices within `tol` of the plane).
// A shadow segment leaving p can meet none of those other triangles nearer to
// p than this, and meets p's own and the coplanar ones only at s = 0 (or, at
// FP32 rounding of their planes, at a grazing angle), so the part of its range
// nearer to p needs no test.  The 64 lanes walk the BVH together with uniform
// control: a child is entered while, for some lane, its box is nearer than
// that lane's nearest triangle so far and does not lie in the lane's plane
// (boxes of a floor or a wall are passed over whole); each lane keeps its own
// minimum.  A lane also tests the triangles of children entered for other
// lanes, and the in-plane test of a box and of its triangles round
// differently, so a value may depend on the wave's other points: a pixel's
// radius is always the one its 8 x 8 tile's wave computes (gather_tile, and
// the dump, which walks the same tiles).  The search stops at the cap (a lane
// with no triangle to consider within it gets the cap, shortened like any
// radius); inactive lanes get 0.
__device__ float free_radius(const DevScene& sc, float cap, float px, float py, float pz, float nx, float ny, float nz, int ex,
                             bool act, int lane)
{
    float tol, margin, cap2;
    free_bounds(sc, cap, &tol, &margin, &cap2);
    // without a unit normal there is no plane to leave: such a point gets 0
    act = act && fmaf(nz, nz, fmaf(ny, ny, nx * nx)) > 0.5f;
    const float4* __restrict__ nodes = sc.nodes;
    const float4* __restrict__ tris = sc.tris;  // identity plane: vertices in (x, y, z) order
    // boxes are padded outward, so a box's distance is below that of any
    // triangle in it by more than FP32 rounding: pruning at best2 is exact
    float best2 = act ? cap2 : -1.f;
    int slot = 0;
    int sp = 0;
    int node = 0;
    const int lead = __builtin_ctzll(ballot(act) | (1ull << 63));
    while (true) {
        const Rec nd = load_rec(nodes, node);
        const int c0 = __float_as_int(nd.q3.x), c1 = __float_as_int(nd.q3.y), kk = __float_as_int(nd.q3.z);
        const float d0 = box_dist2(px, py, pz, nd.q0.x, nd.q0.y, nd.q0.z, nd.q0.w, nd.q2.x, nd.q2.y);
        const float d1 = box_dist2(px, py, pz, nd.q1.x, nd.q1.y, nd.q1.z, nd.q1.w, nd.q2.z, nd.q2.w);
        bool e0 = ballot(d0 < best2 && !box_in_plane(px, py, pz, nx, ny, nz, nd.q0.x, nd.q0.y, nd.q0.z, nd.q0.w, nd.q2.x,
                                                     nd.q2.y, tol)) != 0;
        bool e1 = ballot(d1 < best2 && !box_in_plane(px, py, pz, nx, ny, nz, nd.q1.x, nd.q1.y, nd.q1.z, nd.q1.w, nd.q2.z,
                                                     nd.q2.w, tol)) != 0;
        for (int k = 0; k < 2; ++k) {
            const int cnt = k == 0 ? (kk & 0xffff) : (kk >> 16);
            const bool enter = k == 0 ? e0 : e1;
            if (cnt == 0 || !enter) continue;
            const int first = k == 0 ? c0 : c1;
            for (int i = first; i < first + cnt; ++i) {
                const Rec rec = load_rec(tris, i);
                const bool near = free_tri_near(px, py, pz, rec, best2);
                if (ballot(near) == 0) continue;  // the triangle's box is no nearer than any lane's best
                const float oa = fmaf(nz, rec.q0.z - pz, fmaf(ny, rec.q0.y - py, nx * (rec.q0.x - px)));
                const float ob = fmaf(nz, rec.q1.z - pz, fmaf(ny, rec.q1.y - py, nx * (rec.q1.x - px)));
                const float oc = fmaf(nz, rec.q2.z - pz, fmaf(ny, rec.q2.y - py, nx * (rec.q2.x - px)));
                const bool skip = __float_as_int(rec.q0.w) == ex || fmaxf(fmaxf(fabsf(oa), fabsf(ob)), fabsf(oc)) <= tol;
                if (near && !skip) best2 = fminf(best2, tri_dist2(px, py, pz, rec));
            }
            if (k == 0) e0 = false;
            else e1 = false;
        }
        if (e0 && e1) {
            // both: the one nearer the lead lane first
            const bool first1 = __builtin_amdgcn_readlane(__float_as_int(d1), lead) <
                                __builtin_amdgcn_readlane(__float_as_int(d0), lead);  // non-negative floats: int order
            slot = lane == sp ? (first1 ? c0 : c1) : slot;
            ++sp;
            node = first1 ? c1 : c0;
        } else if (e0) {
            node = c0;
        } else if (e1) {
            node = c1;
        } else {
            if (sp == 0) break;
            --sp;
            node = __builtin_amdgcn_readlane(slot, sp);
        }
    }
    return act ? free_safe(best2, margin) : 0.f;
}

// Any-hit test of a wave's 64 segments o + s d, s in (tlo, thi), walked as
// one packet.  `act` marks the lanes with a ray; ex0 (per lane) and ex1
// (wave-uniform) are the excluded host triangles; rx (per lane) and ry
// (wave-uniform) are the free radii of the segments' ends (0: none), which
// clip each range to s in (max(tlo, rx / |d|), min(thi, 1 - ry / |d|)): no
// triangle the test considers lies nearer an end than its radius.  A segment
// whose clipped range is empty is unblocked without a walk.  Returns, per
// lane, whether its ray is active and unblocked.  All control is
// wave-uniform: `alive` is the mask of unblocked lanes, and the traversal
// stack holds entry i in lane i of `slot`.
template <bool COUNT>
__device__ __forceinline__ bool packet_visible(const DevScene& sc, float ox, float oy, float oz, float dx, float dy, float dz,
                               bool act, float tlo, float thi, int ex0, int ex1, float rx, float ry, int lane,
                               Counters& cnt)
{
    const float il = __builtin_amdgcn_rsqf(dx * dx + dy * dy + dz * dz);  // the gather's r2, computed alike
    tlo = fmaxf(tlo, rx * il);
    thi = fminf(thi, fmaf(-ry, il, 1.0f));
    const bool open = act && !(tlo < thi);  // the whole range lies within the free radii
    act = act && tlo < thi;
    if (ballot(act) == 0) return open;
    // slab distances in units of the segment's range: u = (s - tlo) * us (an
    // approximate reciprocal only scales every distance alike)
    const float us = rcpf(thi - tlo);
    const float ix = safe_inv(dx), iy = safe_inv(dy), iz = safe_inv(dz);
    SlabRay r;
    r.ix = ix * us;
    r.iy = iy * us;
    r.iz = iz * us;
    r.ox = fmaf(ox, ix, tlo) * us;
    r.oy = fmaf(oy, iy, tlo) * us;
    r.oz = fmaf(oz, iz, tlo) * us;
    WtRay wr = wt_ray(ox, oy, oz, dx, dy, dz);
    const float4* __restrict__ nodes = sc.nodes;
    const float4* __restrict__ tris = sc.tris;
    ex1 = __builtin_amdgcn_readfirstlane(ex1);  // uniform by contract; keeps the leaf loop scalar
    const unsigned long long am = ballot(act);
    // one dominant axis for every active lane: triangle records from that
    // axis's plane, whose vertices need no per-lane permutation
    const int kz0 = __builtin_amdgcn_readlane(wr.kz, __builtin_ctzll(am | (1ull << 63)));
    if ((ballot(wr.kz != kz0) & am) == 0) {
        wr.pre = true;
        wr.okx = sel3(ox, oy, oz, wr.kx);
        wr.oky = sel3(ox, oy, oz, wr.ky);
        wr.okz = sel3(ox, oy, oz, wr.kz);
        tris = sc.tris_rot + (size_t)kz0 * kTriStride * sc.n_tris;
    }
    // one sign pattern for every active lane: the slab entry planes are fixed
    const unsigned long long sx = ballot(r.ix < 0.f) & am, sy = ballot(r.iy < 0.f) & am, sz = ballot(r.iz < 0.f) & am;
    const bool uni = (sx == 0 || sx == am) && (sy == 0 || sy == am) && (sz == 0 || sz == am);
    const int oct = uni ? (sx ? 1 : 0) | (sy ? 2 : 0) | (sz ? 4 : 0) : 8;
    // child order: the midpoint of the first active lane's segment
    const int lead = __builtin_ctzll(am | (1ull << 63));
    const int mkx = __builtin_amdgcn_readfirstlane(order_key(__int_as_float(__builtin_amdgcn_readlane(
        __float_as_int(fmaf(0.5f, dx, ox)), lead))));
    const int mky = __builtin_amdgcn_readfirstlane(order_key(__int_as_float(__builtin_amdgcn_readlane(
        __float_as_int(fmaf(0.5f, dy, oy)), lead))));
    const int mkz = __builtin_amdgcn_readfirstlane(order_key(__int_as_float(__builtin_amdgcn_readlane(
        __float_as_int(fmaf(0.5f, dz, oz)), lead))));
    bool vis;
    switch (oct) {
    case 0: vis = traverse<COUNT, 0>(nodes, tris, r, wr, act, tlo, thi, ex0, ex1, mkx, mky, mkz, lane, cnt); break;
    case 1: vis = traverse<COUNT, 1>(nodes, tris, r, wr, act, tlo, thi, ex0, ex1, mkx, mky, mkz, lane, cnt); break;
    case 2: vis = traverse<COUNT, 2>(nodes, tris, r, wr, act, tlo, thi, ex0, ex1, mkx, mky, mkz, lane, cnt); break;
    case 3: vis = traverse<COUNT, 3>(nodes, tris, r, wr, act, tlo, thi, ex0, ex1, mkx, mky, mkz, lane, cnt); break;
    case 4: vis = traverse<COUNT, 4>(nodes, tris, r, wr, act, tlo, thi, ex0, ex1, mkx, mky, mkz, lane, cnt); break;
    case 5: vis = traverse<COUNT, 5>(nodes, tris, r, wr, act, tlo, thi, ex0, ex1, mkx, mky, mkz, lane, cnt); break;
    case 6: vis = traverse<COUNT, 6>(nodes, tris, r, wr, act, tlo, thi, ex0, ex1, mkx, mky, mkz, lane, cnt); break;
    case 7: vis = traverse<COUNT, 7>(nodes, tris, r, wr, act, tlo, thi, ex0, ex1, mkx, mky, mkz, lane, cnt); break;
    default: vis = traverse<COUNT, 8>(nodes, tris, r, wr, act, tlo, thi, ex0, ex1, mkx, mky, mkz, lane, cnt); break;
    }
    return vis || open;
}

// Pixel of lane `tid` in a 16 x 16 tile: each wave64 owns an 8 x 8 quadrant.
__device__ __forceinline__ void tile_pixel(int tid, int bx, int by, int* px, int* py)
{
    int w = tid >> 6, lane = tid & 63;
    *px = bx * 16 + (w & 1) * 8 + (lane & 7);
    *py = by * 16 + (w >> 1) * 8 + (lane >> 3);
}

// Gather of one 8 x 8 pixel tile by a group of `nw` waves (wave `wave` of
// the group takes k = wave, wave + nw, ...), each wave tracing its shadow
// rays as one packet.  The sum of a pixel is fixed in three levels: a wave
// adds its terms in chunks of kChunk VPLs (round r of the wave covers
// k = wave + (r * kChunk + j) * nw, j < kChunk); the rounds fall into kGroups
// groups of consecutive rounds, and the wave adds its chunk sums group by
// group; a group's wave sums are added in wave order, and the group sums in
// group order.  So the result of a pixel depends only on (tile, nw), never on
// what else runs in the launch nor on whether its groups ran in one workgroup
// or in several.  This call covers groups [g0, g1) and returns, in wave 0's
// lanes, the group sums of its range added in order.  `red` (LDS) holds
// (g1 - g0) * nw slots of [3][64].  All waves of the group must call this
// together; `sync` is a barrier over the group.
template <bool COUNT, class Sync>
__device__ __forceinline__ float3 gather_tile(const GatherArgs& a, int tile, int g0, int g1, int wave, int nw, int lane,
                                              float (*red)[3][64], Counters& cnt, unsigned long long& pairs, Sync sync)
{
    const int W = a.gb.width, H = a.gb.height;
    const int tiles_x = (W + 7) >> 3;
    const int px = (tile % tiles_x) * 8 + (lane & 7);
    const int py = (tile / tiles_x) * 8 + (lane >> 3);
    const bool valid = px < W && py < H;
    const int p = py * W + px;
    float x = 0, y = 0, z = 0, nx = 0, ny = 0, nz = 0;
    int tp = -1;
    if (valid) {
        tp = a.gb.tri[p];
        x = a.gb.pos[0][p]; y = a.gb.pos[1][p]; z = a.gb.pos[2][p];
        nx = a.gb.nrm[0][p]; ny = a.gb.nrm[1][p]; nz = a.gb.nrm[2][p];
    }
    const bool active = valid && tp >= 0;
    // free radii of the tile's receivers: wave 0 of the group walks for them, the group reads them from
    // LDS (the slot is free until the group's first round-group sums)
    if (wave == 0) red[0][0][lane] = a.free_ends & 1 ? free_radius(a.scene, kFreeCapTile, x, y, z, nx, ny, nz, tp, active, lane) : 0.f;
    sync();
    const float rx = red[0][0][lane];
    sync();
    const int M = *a.vpls.count;
    const float C = a.g_clamp;
    const float tlo = a.t_eps, thi = 1.0f - a.t_eps;
    const float4* __restrict__ vp = a.vpls.pack;
    const int step = nw * kChunk;
    const int R = (M + step - 1) / step;  // rounds of wave 0 (the most of any wave)
    const bool any = ballot(active) != 0;
    for (int g = g0; g < g1; ++g) {
        float ar = 0.f, ag = 0.f, ab = 0.f;
        const int r1 = (g + 1) * R / kGroups;
        for (int base = wave + g * R / kGroups * step; any && base < r1 * step; base += step) {
            float pr = 0.f, pg = 0.f, pb = 0.f;
            for (int j = 0; j < kChunk; ++j) {
                const int k = base + j * nw;
                if (k >= M) break;
                if (COUNT && active) pairs++;
                const float4 v0 = load_c4(vp, 3 * k), v1 = load_c4(vp, 3 * k + 1);
                float dx = v0.x - x, dy = v0.y - y, dz = v0.z - z;
                float cp = nx * dx + ny * dy + nz * dz;
                float ck = -(v1.x * dx + v1.y * dy + v1.z * dz);
                bool act = active && cp > 0.f && ck > 0.f;
                if (ballot(act) == 0) continue;
                if (COUNT && act) cnt.rays++;
                if (COUNT) {
                    const int n_act = __builtin_popcountll(ballot(act));
                    if (lane == 0) {
                        cnt.packets++;
                        cnt.plane += n_act;
                    }
                }
                float r2 = dx * dx + dy * dy + dz * dz;
                float gt = fminf(C, cp * ck * rcpf(r2 * r2));
                bool vis = packet_visible<COUNT>(a.scene, x, y, z, dx, dy, dz, act, tlo, thi, tp, __float_as_int(v0.w),
                                                 rx, a.free_ends & 2 ? v1.w : 0.f, lane, cnt);
                if (COUNT) {
                    const unsigned long long am = ballot(act), vm = ballot(vis);
                    if (act && !vis) cnt.blocked++;
                    if (lane == 0) {
                        cnt.pk_blocked += vm == 0;
                        cnt.pk_clear += vm == am;
                    }
                }
                if (vis) {
                    const float4 v2 = load_c4(vp, 3 * k + 2);
                    pr = fmaf(v2.x, gt, pr);
                    pg = fmaf(v2.y, gt, pg);
                    pb = fmaf(v2.z, gt, pb);
                }
            }
            ar += pr;
            ag += pg;
            ab += pb;
        }
        const int slot = (g - g0) * nw + wave;
        red[slot][0][lane] = ar;
        red[slot][1][lane] = ag;
        red[slot][2][lane] = ab;
    }
    sync();
    float3 S = make_float3(0.f, 0.f, 0.f);
    if (wave == 0) {
        for (int g = 0; g < g1 - g0; ++g) {
            float sr = 0.f, sg = 0.f, sb = 0.f;
            for (int w = 0; w < nw; ++w) {
                sr += red[g * nw + w][0][lane];
                sg += red[g * nw + w][1][lane];
                sb += red[g * nw + w][2][lane];
            }
            S.x += sr;
            S.y += sg;
            S.z += sb;
        }
    }
    sync();
    return S;
}

// Radiance of the tile's pixel in `lane` from its summed terms: albedo / pi
// times the sum on a surface hit, 0 on a miss.
__device__ __forceinline__ void tile_out(const GatherArgs& a, int tile, int lane, float3 S)
{
    const int W = a.gb.width, H = a.gb.height;
    const int tiles_x = (W + 7) >> 3;
    const int px = (tile % tiles_x) * 8 + (lane & 7);
    const int py = (tile / tiles_x) * 8 + (lane >> 3);
    if (px >= W || py >= H) return;
    const int p = py * W + px;
    const bool active = a.gb.tri[p] >= 0;
    const float s = kInvPi;
    a.out[0][p] = active ? a.gb.alb[0][p] * s * S.x : 0.f;
    a.out[1][p] = active ? a.gb.alb[1][p] * s * S.y : 0.f;
    a.out[2][p] = active ? a.gb.alb[2][p] * s * S.z : 0.f;
}

// Pixel blocks of a view: G = 1, 2 or 4 tiles of 8 x 8 pixels (1 x 1, 2 x 1 or
// 2 x 2 tiles), row-major over the view's block grid.
__host__ __device__ __forceinline__ int block_cols(int G) { return G == 1 ? 1 : 2; }
__host__ __device__ __forceinline__ int block_rows(int G) { return G == 4 ? 2 : 1; }
__host__ __device__ __forceinline__ int view_blocks(int W, int H, int G)
{
    const int tx = (W + 7) >> 3, ty = (H + 7) >> 3;
    return ((tx + block_cols(G) - 1) / block_cols(G)) * ((ty + block_rows(G) - 1) / block_rows(G));
}

// Tile (row-major index over the view's 8 x 8 tiles) of sub-tile i of block
// b, or -1 where the block hangs over the view's edge.
__device__ __forceinline__ int block_tile(int b, int i, int G, int W, int H)
{
    const int tx_n = (W + 7) >> 3, ty_n = (H + 7) >> 3;
    const int bw = block_cols(G), bh = block_rows(G);
    const int bx_n = (tx_n + bw - 1) / bw;
    const int tx = (b % bx_n) * bw + i % bw, ty = (b / bx_n) * bh + i / bw;
    return tx < tx_n && ty < ty_n ? ty * tx_n + tx : -1;
}

template <bool COUNT>
__device__ __forceinline__ void flush_counters(unsigned long long* out, const Counters& cnt, unsigned long long pairs,
                                               int lane)
{
    if (!COUNT) return;
    const unsigned long long v[kCounters] = {pairs, cnt.rays, cnt.nodes, cnt.tris, cnt.packets, cnt.psteps, cnt.plane,
                                             cnt.ptris, cnt.rides, cnt.both, cnt.pops, cnt.pk_blocked, cnt.pk_clear,
                                             cnt.blocked};
    for (int c = 0; c < kCounters; ++c) {
        unsigned long long sum = v[c];
        for (int off = 32; off > 0; off >>= 1) sum += __shfl_down(sum, off, 64);
        if (lane == 0) atomicAdd(&out[c], sum);
    }
}

struct BlockSync {
    __device__ void operator()() const { __syncthreads(); }
};

// The workgroup barriers of one gather_tile call (two around the free radii,
// two around the group sums), for the waves of a group that has no tile.
__device__ __forceinline__ void tile_skip_barriers()
{
    __syncthreads();
    __syncthreads();
    __syncthreads();
    __syncthreads();
}

// Persistent gather of one view: each workgroup (G tile groups of w waves,
// one VPL slice each) claims work items from a device counter until none is
// left, so the tiles' uneven costs spread over all CUs of all XCDs (a fixed
// tile per workgroup leaves whole XCDs idle: the hardware deals workgroups to
// the XCDs round robin, whatever their cost).  An item is a pixel block of G
// tiles, each gathered by its own group.  Items [0, split_full) are whole
// blocks; the last split_count blocks are claimed as kGroups items of one
// round group each, so the launch ends on items a kGroups-th of a block long
// instead of idling behind its last whole blocks (on a 512 x 512 view of
// 4,096 VPLs the launch takes 5% less time).  A split item stores each of its
// tiles' group sums in split_part; k_gather_split_finish (the next kernel on
// the stream) adds a tile's group sums in group order -- the whole tile's own
// order, so a split tile's result is bit for bit the unsplit one.  No
// workgroup waits for another, and every workgroup reaches the exit.
template <bool COUNT>
__device__ __forceinline__ void gather_persistent(const GatherArgs& a, unsigned int* __restrict__ counter)
{
    extern __shared__ float s_dyn[];  // kGroups * G * w slots of [3][64]
    float (*s_red)[3][64] = reinterpret_cast<float (*)[3][64]>(s_dyn);
    __shared__ int s_item;
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int nw = a.waves_per_tile, G = a.px_tiles;
    const int grp = wave / nw, wg = wave % nw;
    const int W = a.gb.width, H = a.gb.height;
    const int full = a.split_full;
    const int total = full + a.split_count * kGroups;
    Counters cnt;
    unsigned long long pairs = 0;
    while (true) {
        if (threadIdx.x == 0) s_item = (int)atomicAdd(counter, 1u);
        __syncthreads();
        const int item = __builtin_amdgcn_readfirstlane(s_item);  // an LDS value is uniform here
        __syncthreads();
        if (item >= total) break;
        // a whole block, or split slot si: round group si % kGroups of block full + si / kGroups
        const bool whole = item < full;
        const int si = whole ? 0 : item - full;
        const int g = si % kGroups;
        const int blk = whole ? item : full + si / kGroups;
        const int tile = block_tile(blk, grp, G, W, H);
        float (*red)[3][64] = s_red + grp * kGroups * nw;
        if (tile < 0) {  // every wave takes part in the tile's barriers
            tile_skip_barriers();
            continue;
        }
        const float3 S = gather_tile<COUNT>(a, tile, whole ? 0 : g, whole ? kGroups : g + 1, wg, nw, lane, red, cnt,
                                            pairs, BlockSync());
        if (wg != 0) continue;
        if (whole) {
            tile_out(a, tile, lane, S);
        } else {
            float* part = a.split_part + ((size_t)(si / kGroups * G + grp) * kGroups + g) * 192;
            part[lane] = S.x;
            part[64 + lane] = S.y;
            part[128 + lane] = S.z;
        }
    }
    flush_counters<COUNT>(a.counters, cnt, pairs, lane);
}

// The plain gather is held to 8 waves per SIMD (its few scalar spills cost
// less than a lost wave); the instrumented one keeps its registers.
__global__ __launch_bounds__(kGatherMaxThreads) __attribute__((amdgpu_waves_per_eu(8))) void k_gather(
    GatherArgs a, unsigned int* __restrict__ counter)
{
    gather_persistent<false>(a, counter);
}

__global__ __launch_bounds__(kGatherMaxThreads) void k_gather_counted(GatherArgs a, unsigned int* __restrict__ counter)
{
    gather_persistent<true>(a, counter);
}

// One wave per tile of the split blocks of the preceding gather: its group
// sums added in group order, then the pixel's radiance.
__global__ __launch_bounds__(64) void k_gather_split_finish(GatherArgs a)
{
    const int st = blockIdx.x, lane = threadIdx.x;
    const int G = a.px_tiles;
    const int tile = block_tile(a.split_full + st / G, st % G, G, a.gb.width, a.gb.height);
    if (tile < 0) return;  // the whole wave: sub-tile over the view's edge
    const float* q = a.split_part + (size_t)st * kGroups * 192;
    float3 T = make_float3(0.f, 0.f, 0.f);
    for (int h = 0; h < kGroups; ++h) {
        T.x += q[h * 192 + lane];
        T.y += q[h * 192 + 64 + lane];
        T.z += q[h * 192 + 128 + lane];
    }
    tile_out(a, tile, lane, T);
}

// Persistent gather over many views.  Each workgroup of BW waves claims
// work items from a device counter until none is left (every workgroup
// reaches the exit).  The workgroup holds g = BW / w_v tile groups of w_v
// waves; item j of view v covers its pixel blocks [j * g / G, (j + 1) * g / G)
// of G tiles each (group i takes sub-tile i % G of block j * g / G + i / G).
template <int BW>
__global__ __launch_bounds__(64 * BW) __attribute__((amdgpu_waves_per_eu(8))) void k_gather_batch(
    const BatchTable* __restrict__ tab, const GatherArgs* __restrict__ views, unsigned int* __restrict__ counter)
{
    __shared__ float s_red[kGroups * BW][3][64];
    __shared__ int s_item;
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int n_views = tab->n_views;
    const int total = tab->prefix[n_views];
    Counters cnt;
    unsigned long long pairs = 0;
    while (true) {
        if (threadIdx.x == 0) s_item = (int)atomicAdd(counter, 1u);
        __syncthreads();
        const int item = __builtin_amdgcn_readfirstlane(s_item);  // an LDS value is uniform here
        __syncthreads();
        if (item >= total) break;
        int lo = 0, hi = n_views;  // view: last v with prefix[v] <= item
        while (hi - lo > 1) {
            int mid = (lo + hi) >> 1;
            if (tab->prefix[mid] <= item) lo = mid; else hi = mid;
        }
        const GatherArgs& a = views[lo];
        const int w = tab->waves[lo];
        const int groups = BW / w;
        const int group = wave / w;
        const int G = a.px_tiles;
        const int blk = (item - tab->prefix[lo]) * (groups / G) + group / G;
        // every wave takes part in the tile's barriers, including groups past the last block
        const int t = blk < view_blocks(a.gb.width, a.gb.height, G) ? block_tile(blk, group % G, G, a.gb.width,
                                                                                  a.gb.height)
                                                                      : -1;
        if (t >= 0) {
            const float3 S = gather_tile<false>(a, t, 0, kGroups, wave % w, w, lane, s_red + group * kGroups * w, cnt,
                                                pairs, BlockSync());
            if (wave % w == 0) tile_out(a, t, lane, S);
        } else {
            tile_skip_barriers();
        }
    }
}

// Zero the work counter (a fill kernel: graph replays clear it reliably).
__global__ void k_reset_counter(unsigned int* counter) { *counter = 0u; }

// One lane per listed pixel; a wave walks the VPLs and records, per lane,
// bit k % 32 of word k / 32 = V(x_p, y_k) for every pair (no geometry-term
// culling), with the gather's own packet traversal.
__global__ __launch_bounds__(BLOCK) void k_vis_dump(VisDumpArgs a)
{
    const int gid = blockIdx.x * BLOCK + threadIdx.x;
    const int lane = threadIdx.x & 63;
    const bool in = gid < a.n_px;
    int p = in ? a.pixels[gid] : -1;
    if (p >= a.gb.width * a.gb.height) p = -1;  // the pixel list lives on the device: checked here
    const int tp = p >= 0 ? a.gb.tri[p] : -1;
    const bool ok = p >= 0 && tp >= 0;
    float x = 0, y = 0, z = 0, nx = 0, ny = 0, nz = 0;
    if (ok) {
        x = a.gb.pos[0][p]; y = a.gb.pos[1][p]; z = a.gb.pos[2][p];
        nx = a.gb.nrm[0][p]; ny = a.gb.nrm[1][p]; nz = a.gb.nrm[2][p];
    }
    // the gather's clipping with its free radii: a pixel's radius is the one its 8 x 8 tile's wave
    // computes, so the dump walks each tile its pixels fall in with that tile's 64 pixels, lane for lane
    const int W = a.gb.width, H = a.gb.height, tiles_x = (W + 7) >> 3;
    const int my_tile = p >= 0 ? (p / W >> 3) * tiles_x + ((p % W) >> 3) : -1;
    const int my_pos = p >= 0 ? ((p % W) & 7) | ((p / W & 7) << 3) : 0;
    float rx = 0.f;
    unsigned long long todo = a.free_ends & 1 ? ballot(ok) : 0ull;
    while (todo) {
        const int T = __builtin_amdgcn_readlane(my_tile, __builtin_ctzll(todo));
        const int qx = (T % tiles_x) * 8 + (lane & 7), qy = (T / tiles_x) * 8 + (lane >> 3);
        const bool qv = qx < W && qy < H;
        const int q = qy * W + qx;
        int qt = -1;
        float qpx = 0, qpy = 0, qpz = 0, qnx = 0, qny = 0, qnz = 0;
        if (qv) {
            qt = a.gb.tri[q];
            qpx = a.gb.pos[0][q]; qpy = a.gb.pos[1][q]; qpz = a.gb.pos[2][q];
            qnx = a.gb.nrm[0][q]; qny = a.gb.nrm[1][q]; qnz = a.gb.nrm[2][q];
        }
        const float r = free_radius(a.scene, kFreeCapTile, qpx, qpy, qpz, qnx, qny, qnz, qt, qv && qt >= 0, lane);
        const float mine = __shfl(r, my_pos, 64);
        const bool here = ok && my_tile == T;
        if (here) rx = mine;
        todo &= ~ballot(here);
    }
    const int M = *a.vpls.count;
    const float4* __restrict__ vp = a.vpls.pack;
    Counters cnt;
    for (int w = 0; w < a.words; ++w) {
        uint32_t bits = 0;
        for (int b = 0; b < 32; ++b) {
            int k = w * 32 + b;
            if (k >= M) break;
            const float4 v0 = load_c4(vp, 3 * k);
            const float ry = a.free_ends & 2 ? load_c4(vp, 3 * k + 1).w : 0.f;
            bool vis = false;
            if (ballot(ok) != 0)
                vis = packet_visible<false>(a.scene, x, y, z, v0.x - x, v0.y - y, v0.z - z, ok, a.t_eps,
                                            1.0f - a.t_eps, tp, __float_as_int(v0.w), rx, ry, lane, cnt);
            if (vis) bits |= 1u << b;
        }
        if (in) a.bits[(size_t)gid * a.words + w] = bits;
    }
}

// Direct term L_e(y) of eq. (1) with the light model of eq. (2): per pixel
// (albedo / pi) * Phi * G, G = sum over the light's samples y_j of the
// unoccluded max(0, n.w) / (4 pi r^3) (point light) or max(0, n.w)
// max(0, -n_l.w) / (16 pi r^4) (quad cells), w = y_j - x, r = |w|.  One wave
// per 8 x 8 tile; the 64 shadow rays to one sample form one packet, samples
// summed in order.
__global__ __launch_bounds__(BLOCK) void k_direct(DirectArgs a)
{
    const int lane = threadIdx.x & 63;
    const int W = a.gb.width, H = a.gb.height;
    const int tiles_x = (W + 7) >> 3, tiles = tiles_x * ((H + 7) >> 3);
    const int tile = blockIdx.x * (BLOCK / 64) + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    if (tile >= tiles) return;  // the whole wave
    const int px = (tile % tiles_x) * 8 + (lane & 7), py = (tile / tiles_x) * 8 + (lane >> 3);
    const bool in = px < W && py < H;
    const int p = py * W + px;
    int tp = -1;
    float x = 0, y = 0, z = 0, nx = 0, ny = 0, nz = 0;
    if (in) {
        tp = a.gb.tri[p];
        x = a.gb.pos[0][p]; y = a.gb.pos[1][p]; z = a.gb.pos[2][p];
        nx = a.gb.nrm[0][p]; ny = a.gb.nrm[1][p]; nz = a.gb.nrm[2][p];
    }
    const bool valid = in && tp >= 0;
    const bool quad = a.light.kind != 0;
    const float tlo = a.t_eps, thi = 1.0f - a.t_eps;
    Counters cnt;
    float G = 0.f;
    for (int j = 0; j < a.light.n_samples; ++j) {
        const float wx = a.light.samples[j][0] - x, wy = a.light.samples[j][1] - y, wz = a.light.samples[j][2] - z;
        const float r2 = fmaf(wz, wz, fmaf(wy, wy, wx * wx));
        const float cx = fmaf(nz, wz, fmaf(ny, wy, nx * wx));
        const float cl = quad ? -fmaf(a.light.nl[2], wz, fmaf(a.light.nl[1], wy, a.light.nl[0] * wx)) : 1.0f;
        const bool act = valid && cx > 0.f && cl > 0.f;
        if (ballot(act) == 0) continue;
        const float g = quad ? (cx * cl) * rcpf(r2 * r2) : cx * rcpf(r2 * sqrtf(r2));
        const bool vis = packet_visible<false>(a.scene, x, y, z, wx, wy, wz, act, tlo, thi, tp, -1, 0.f, 0.f, lane, cnt);
        if (vis) G += g;
    }
    G *= quad ? 1.0f / (16.0f * 3.14159265358979323846f) : 1.0f / (4.0f * 3.14159265358979323846f);
    if (in) {
        for (int c = 0; c < 3; ++c) a.out[c][p] = valid ? a.gb.alb[c][p] * kInvPi * (a.light.power[c] * G) : 0.f;
    }
}

// Closest hit, t in (0, inf); ties go to the smaller original triangle index.
__global__ __launch_bounds__(BLOCK) void k_gbuffer(GBufferArgs a)
{
    __shared__ int s_stack[kStack * BLOCK];
    const int tid = threadIdx.x;
    int px, py;
    tile_pixel(tid, blockIdx.x, blockIdx.y, &px, &py);
    if (px >= a.width || py >= a.height) return;
    const int p = py * a.width + px;
    float sx = (2.0f * ((float)px + 0.5f) / (float)a.width - 1.0f) * a.tx;
    float sy = (1.0f - 2.0f * ((float)py + 0.5f) / (float)a.height) * a.th;
    float dx = a.f[0] + sx * a.r[0] + sy * a.u[0];
    float dy = a.f[1] + sx * a.r[1] + sy * a.u[1];
    float dz = a.f[2] + sx * a.r[2] + sy * a.u[2];
    float ox = a.eye[0], oy = a.eye[1], oz = a.eye[2];
    SlabRay r;
    r.ix = safe_inv(dx);
    r.iy = safe_inv(dy);
    r.iz = safe_inv(dz);
    r.ox = ox * r.ix;
    r.oy = oy * r.iy;
    r.oz = oz * r.iz;
    const WtRay wr = wt_ray(ox, oy, oz, dx, dy, dz);
    const float4* __restrict__ nodes = a.scene.nodes;
    const float4* __restrict__ tris = a.scene.tris;
    int* stack = s_stack + tid;
    int sp = 0, node = 0;
    float best = __builtin_inff();
    float bu = 0.f, bv = 0.f;
    int bid = -1, bi = -1;
    while (true) {
        float4 n0 = nodes[4 * node], n1 = nodes[4 * node + 1], n2 = nodes[4 * node + 2], n3f = nodes[4 * node + 3];
        int c0 = __float_as_int(n3f.x), c1 = __float_as_int(n3f.y);
        const int kk = __float_as_int(n3f.z);
        int k0 = kk & 0xffff, k1 = kk >> 16;
        float lo0, hi0, lo1, hi1;
        child_boxes(n0, n1, n2, r, 0.0f, best, &lo0, &hi0, &lo1, &hi1);
        bool h0 = lo0 <= hi0;
        bool h1 = lo1 <= hi1;
        for (int c = 0; c < 2; ++c) {
            bool h = c == 0 ? h0 : h1;
            int first = c == 0 ? c0 : c1, count = c == 0 ? k0 : k1;
            if (h && count > 0) {
                for (int i = first; i < first + count; ++i) {
                    float t, u, v;
                    int id;
                    bool ok = tri_hit32(load_rec(tris, i), wr, 0.0f, __builtin_inff(), &t, &u, &v, &id);
                    if (ok && (t < best || (t == best && id < bid))) {
                        best = t; bu = u; bv = v; bid = id; bi = i;
                    }
                }
                if (c == 0) h0 = false; else h1 = false;
            }
        }
        if (h0 && h1) {
            bool near0 = lo0 <= lo1;
            stack[sp * BLOCK] = near0 ? c1 : c0;
            ++sp;
            node = near0 ? c0 : c1;
        } else if (h0) {
            node = c0;
        } else if (h1) {
            node = c1;
        } else {
            bool found = false;
            while (sp > 0) {
                --sp;
                node = stack[sp * BLOCK];
                found = true;
                break;
            }
            if (!found) break;
        }
    }
    a.tri[p] = bid;
    if (bid < 0) {
        for (int c = 0; c < 3; ++c) { a.pos[c][p] = 0.f; a.nrm[c][p] = 0.f; a.alb[c][p] = 0.f; }
        return;
    }
    const float4 va = tris[kTriStride * bi], vb = tris[kTriStride * bi + 1], vc = tris[kTriStride * bi + 2];
    const float bw = 1.0f - bu - bv;
    a.pos[0][p] = bw * va.x + bu * vb.x + bv * vc.x;
    a.pos[1][p] = bw * va.y + bu * vb.y + bv * vc.y;
    a.pos[2][p] = bw * va.z + bu * vb.z + bv * vc.z;
    float4 n = a.scene.normals[bid];
    a.nrm[0][p] = n.x; a.nrm[1][p] = n.y; a.nrm[2][p] = n.z;
    a.alb[0][p] = a.scene.albedo[3 * bid];
    a.alb[1][p] = a.scene.albedo[3 * bid + 1];
    a.alb[2][p] = a.scene.albedo[3 * bid + 2];
}

// Interleave the SoA planes of a VPL set into the gather layout.
// The gather's VPL records; with a scene, each VPL's free radius in that
// scene goes to the .w of its second record (else 0).  Every lane of a wave
// takes part in the radius walk.
// The gather's VPL records of a set with no scene (free radius 0), one thread per VPL.
__global__ __launch_bounds__(BLOCK) void k_pack_vpls_plain(DevVpls v)
{
    const int i = blockIdx.x * BLOCK + threadIdx.x;
    if (i >= *v.count || i >= v.capacity) return;
    v.pack[3 * i] = make_float4(v.px[i], v.py[i], v.pz[i], __int_as_float(v.tri[i]));
    v.pack[3 * i + 1] = make_float4(v.nx[i], v.ny[i], v.nz[i], 0.f);
    v.pack[3 * i + 2] = make_float4(v.ir[i], v.ig[i], v.ib[i], 0.f);
}

// The gather's VPL records, one wave per VPL; with a scene, the VPL's free
// radius in that scene goes to the .w of its second record (else 0).  Lane 0
// alone drives the radius walk (the other lanes are idle in it), so the value
// depends on the VPL alone, and with one wave per VPL the short, latency-bound
// walks run side by side over the whole device.
__global__ __launch_bounds__(64) void k_pack_vpls(DevScene sc, DevVpls v, int with_radius)
{
    const int i = blockIdx.x;
    if (i >= *v.count || i >= v.capacity) return;  // the whole wave
    const int lane = threadIdx.x;
    const float px = v.px[i], py = v.py[i], pz = v.pz[i];
    const float nx = v.nx[i], ny = v.ny[i], nz = v.nz[i];
    const int tri = v.tri[i];
    const float r = with_radius ? free_radius(sc, kFreeCapVpl, px, py, pz, nx, ny, nz, tri, lane == 0, lane) : 0.f;
    if (lane == 0) {
        v.pack[3 * i] = make_float4(px, py, pz, __int_as_float(tri));
        v.pack[3 * i + 1] = make_float4(nx, ny, nz, r);
        v.pack[3 * i + 2] = make_float4(v.ir[i], v.ig[i], v.ib[i], 0.f);
    }
}

}  // namespace

hipError_t launch_pack_vpls(const DevScene* sc, const DevVpls& v, hipStream_t s)
{
    if (v.capacity == 0) return hipSuccess;
    if (sc) hipLaunchKernelGGL(k_pack_vpls, dim3(v.capacity), dim3(64), 0, s, *sc, v, 1);
    else hipLaunchKernelGGL(k_pack_vpls_plain, dim3((v.capacity + BLOCK - 1) / BLOCK), dim3(BLOCK), 0, s, v);
    return hipGetLastError();
}

// LDS of a single-view gather workgroup of `waves` waves: kGroups slots of
// [3][64] floats per wave (a whole tile's group sums).
static size_t gather_lds_bytes(int waves) { return (size_t)kGroups * waves * 3 * 64 * sizeof(float); }

int gather_view_blocks(int width, int height, int px_tiles) { return view_blocks(width, height, px_tiles); }

hipError_t gather_occupancy(int waves, bool counted, int* blocks_per_cu)
{
    if (waves < 1 || waves > kGatherMaxWaves || (waves & (waves - 1))) return hipErrorInvalidValue;
    const size_t lds = gather_lds_bytes(waves);
    return counted ? hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, k_gather_counted, 64 * waves, lds)
                   : hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, k_gather, 64 * waves, lds);
}

int gather_split_floats_per_tile() { return kGroups * 3 * 64; }

// Device address of `scratch` per device.  In host code the array's name is
// only a host-side handle, so launches take the address looked up here.
namespace {
constexpr int kMaxDevices = 256;
std::mutex g_scratch_mu;
void* g_scratch_addr[kMaxDevices] = {};
}  // namespace

hipError_t gather_scratch_setup(int device)
{
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (g_scratch_addr[device]) return hipSuccess;
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!p) return hipErrorInvalidSymbol;
    g_scratch_addr[device] = p;
    return hipSuccess;
}

void* gather_scratch_address(int device)
{
    if (device < 0 || device >= kMaxDevices) return nullptr;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    return g_scratch_addr[device];
}

size_t gather_scratch_bytes() { return kScratchBytes; }

int gather_scratch_split_cap() { return kScratchSplitTiles; }

hipError_t launch_gather_scratch(const GatherArgs& a, void* scr, int blocks, hipStream_t s)
{
    if (!scr) return hipErrorInvalidValue;
    GatherArgs b = a;
    b.split_cap = kScratchSplitTiles;
    b.split_part = reinterpret_cast<float*>(static_cast<unsigned char*>(scr) + 256);
    return launch_gather(b, false, static_cast<unsigned int*>(scr), blocks, s);
}

hipError_t launch_gather(const GatherArgs& a, bool counted, unsigned int* counter, int blocks, hipStream_t s)
{
    const int G = a.px_tiles;
    const int waves = a.waves_per_tile * G;
    if (G != 1 && G != 2 && G != 4) return hipErrorInvalidValue;
    if (waves < 1 || waves > kGatherMaxWaves || (waves & (waves - 1)) || !counter || blocks < 1 ||
        a.split_cap < 0 || (a.split_cap > 0 && !a.split_part))
        return hipErrorInvalidValue;
    const int nblk = view_blocks(a.gb.width, a.gb.height, G);
    const int nb = blocks < nblk ? blocks : nblk;
    // the last kSplitRounds rounds of blocks (kSplitRounds per workgroup, at
    // most split_cap tiles) are claimed by round group, in views of at least
    // 2 kSplitRounds rounds; smaller views keep whole blocks (they have no
    // long tail, and quarter blocks would only add per-item work)
    GatherArgs b = a;
    b.split_count = nblk >= 2 * kSplitRounds * nb ? std::min(nb * kSplitRounds, a.split_cap / G) : 0;
    b.split_full = nblk - b.split_count;
    dim3 grid(nb), block(64 * waves);
    const size_t lds = gather_lds_bytes(waves);
    hipLaunchKernelGGL(k_reset_counter, dim3(1), dim3(1), 0, s, counter);
    if (counted)
        hipLaunchKernelGGL(k_gather_counted, grid, block, lds, s, b, counter);
    else
        hipLaunchKernelGGL(k_gather, grid, block, lds, s, b, counter);
    if (b.split_count > 0) hipLaunchKernelGGL(k_gather_split_finish, dim3(b.split_count * G), dim3(64), 0, s, b);
    return hipGetLastError();
}

hipError_t launch_gather_batch(const BatchTable* tab, const GatherArgs* views, unsigned int* counter, int blocks,
                               int block_waves, hipStream_t s)
{
    if (block_waves != kBatchBlockWaves && block_waves != kBatchWideWaves) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_reset_counter, dim3(1), dim3(1), 0, s, counter);
    if (block_waves == kBatchWideWaves)
        hipLaunchKernelGGL(k_gather_batch<kBatchWideWaves>, dim3(blocks), dim3(64 * kBatchWideWaves), 0, s, tab, views,
                           counter);
    else
        hipLaunchKernelGGL(k_gather_batch<kBatchBlockWaves>, dim3(blocks), dim3(64 * kBatchBlockWaves), 0, s, tab,
                           views, counter);
    return hipGetLastError();
}

hipError_t gather_batch_occupancy(int block_waves, int* blocks_per_cu)
{
    if (block_waves == kBatchWideWaves)
        return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, k_gather_batch<kBatchWideWaves>,
                                                            64 * kBatchWideWaves, 0);
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, k_gather_batch<kBatchBlockWaves>,
                                                        64 * kBatchBlockWaves, 0);
}

hipError_t launch_vis_dump(const VisDumpArgs& a, hipStream_t s)
{
    if (a.n_px == 0 || a.words == 0) return hipSuccess;
    dim3 grid((unsigned)((a.n_px + BLOCK - 1) / BLOCK));
    hipLaunchKernelGGL(k_vis_dump, grid, dim3(BLOCK), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_direct(const DirectArgs& a, hipStream_t s)
{
    const int tiles = ((a.gb.width + 7) / 8) * ((a.gb.height + 7) / 8);
    hipLaunchKernelGGL(k_direct, dim3((tiles + BLOCK / 64 - 1) / (BLOCK / 64)), dim3(BLOCK), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_gbuffer(const GBufferArgs& a, hipStream_t s)
{
    dim3 grid((a.width + 15) / 16, (a.height + 15) / 16);
    hipLaunchKernelGGL(k_gbuffer, grid, dim3(BLOCK), 0, s, a);
    return hipGetLastError();
}

}  // namespace vplg
