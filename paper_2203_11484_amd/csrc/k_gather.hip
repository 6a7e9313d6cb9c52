// FP32 kernels of the VPL gather (eq. (1) without the direct term), its
// visibility dump, and the primary-ray G-buffer.
//
// Every shadow ray is the segment x + s (y - x), s in (t_eps, 1 - t_eps),
// tested against the BVH with both host triangles excluded; occlusion is
// two-sided and emitters occlude.  Traversal stacks live in LDS, one column
// per lane (entry i of lane l at [i * BLOCK + l]: consecutive lanes hit
// consecutive banks).
#include "vplg_impl.h"

namespace vplg {

namespace {

constexpr int BLOCK = 256;     // 4 wave64 per workgroup
constexpr int TILE_V = 256;    // VPLs staged in LDS per tile
constexpr float kInvPi = 0.318309886183790671538f;

__device__ __forceinline__ float rcpf(float x) { return __builtin_amdgcn_rcpf(x); }

__device__ __forceinline__ float safe_inv(float d)
{
    // A zero direction component would turn the slab test into 0 * inf; a
    // tiny signed value keeps the slab unbounded on that axis instead.
    return rcpf(fabsf(d) > 1e-30f ? d : copysignf(1e-30f, d));
}

struct Counters {
    unsigned long long rays = 0, nodes = 0, tris = 0;
};

// Moller-Trumbore against leaf-ordered triangle i; returns the hit parameter
// in *t.  d2 = |d|^2: rays within kParallelTau of the triangle's plane miss.
__device__ __forceinline__ bool tri_hit32(const float4* __restrict__ tris, int i, float ox, float oy, float oz,
                                          float dx, float dy, float dz, float d2, float tlo, float thi, int ex0,
                                          int ex1, float* tout, float* uout, float* vout, int* idout)
{
    float4 a = tris[3 * i];
    float4 e1 = tris[3 * i + 1];
    float4 e2 = tris[3 * i + 2];
    int id = __float_as_int(a.w);
    float px = dy * e2.z - dz * e2.y;
    float py = dz * e2.x - dx * e2.z;
    float pz = dx * e2.y - dy * e2.x;
    float det = e1.x * px + e1.y * py + e1.z * pz;
    float inv = rcpf(det);
    float tx = ox - a.x, ty = oy - a.y, tz = oz - a.z;
    float u = (tx * px + ty * py + tz * pz) * inv;
    float qx = ty * e1.z - tz * e1.y;
    float qy = tz * e1.x - tx * e1.z;
    float qz = tx * e1.y - ty * e1.x;
    float v = (dx * qx + dy * qy + dz * qz) * inv;
    float t = (e2.x * qx + e2.y * qy + e2.z * qz) * inv;
    *tout = t;
    *uout = u;
    *vout = v;
    *idout = id;
    return u >= 0.f && v >= 0.f && u + v <= 1.f && t > tlo && t < thi && id != ex0 && id != ex1 &&
           det * det > e2.w * d2;
}

struct SlabRay {
    float ix, iy, iz, ox, oy, oz;  // inverse direction and origin * inverse
};

__device__ __forceinline__ void child_boxes(const float4& n0, const float4& n1, const float4& n2, const SlabRay& r,
                                            float tlo, float thi, float* lo0, float* hi0, float* lo1, float* hi1)
{
    float a0 = fmaf(n0.x, r.ix, -r.ox), a1 = fmaf(n0.y, r.ix, -r.ox);
    float b0 = fmaf(n0.z, r.iy, -r.oy), b1 = fmaf(n0.w, r.iy, -r.oy);
    float c0 = fmaf(n2.x, r.iz, -r.oz), c1 = fmaf(n2.y, r.iz, -r.oz);
    *lo0 = fmaxf(fmaxf(fminf(a0, a1), fminf(b0, b1)), fmaxf(fminf(c0, c1), tlo));
    *hi0 = fminf(fminf(fmaxf(a0, a1), fmaxf(b0, b1)), fminf(fmaxf(c0, c1), thi));
    float d0 = fmaf(n1.x, r.ix, -r.ox), d1 = fmaf(n1.y, r.ix, -r.ox);
    float e0 = fmaf(n1.z, r.iy, -r.oy), e1 = fmaf(n1.w, r.iy, -r.oy);
    float f0 = fmaf(n2.z, r.iz, -r.oz), f1 = fmaf(n2.w, r.iz, -r.oz);
    *lo1 = fmaxf(fmaxf(fminf(d0, d1), fminf(e0, e1)), fmaxf(fminf(f0, f1), tlo));
    *hi1 = fminf(fminf(fmaxf(d0, d1), fmaxf(e0, e1)), fminf(fmaxf(f0, f1), thi));
}

// Any hit on the segment o + s d, s in (tlo, thi), skipping triangles ex0/ex1.
template <bool COUNT>
__device__ bool occluded(const DevScene& sc, float ox, float oy, float oz, float dx, float dy, float dz, float tlo,
                         float thi, int ex0, int ex1, int* __restrict__ stack, Counters& cnt)
{
    SlabRay r;
    r.ix = safe_inv(dx);
    r.iy = safe_inv(dy);
    r.iz = safe_inv(dz);
    r.ox = ox * r.ix;
    r.oy = oy * r.iy;
    r.oz = oz * r.iz;
    const float d2 = dx * dx + dy * dy + dz * dz;
    const float4* __restrict__ nodes = sc.nodes;
    const float4* __restrict__ tris = sc.tris;
    int sp = 0;
    int node = 0;
    while (true) {
        float4 n0 = nodes[4 * node];
        float4 n1 = nodes[4 * node + 1];
        float4 n2 = nodes[4 * node + 2];
        float4 n3f = nodes[4 * node + 3];
        int c0 = __float_as_int(n3f.x), c1 = __float_as_int(n3f.y);
        int k0 = __float_as_int(n3f.z), k1 = __float_as_int(n3f.w);
        if (COUNT) cnt.nodes++;
        float lo0, hi0, lo1, hi1;
        child_boxes(n0, n1, n2, r, tlo, thi, &lo0, &hi0, &lo1, &hi1);
        bool h0 = lo0 <= hi0 && c0 >= 0;
        bool h1 = lo1 <= hi1 && c1 >= 0;
        if (h0 && k0 > 0) {
            for (int i = c0; i < c0 + k0; ++i) {
                float t, u, v;
                int id;
                if (COUNT) cnt.tris++;
                if (tri_hit32(tris, i, ox, oy, oz, dx, dy, dz, d2, tlo, thi, ex0, ex1, &t, &u, &v, &id)) return true;
            }
            h0 = false;
        }
        if (h1 && k1 > 0) {
            for (int i = c1; i < c1 + k1; ++i) {
                float t, u, v;
                int id;
                if (COUNT) cnt.tris++;
                if (tri_hit32(tris, i, ox, oy, oz, dx, dy, dz, d2, tlo, thi, ex0, ex1, &t, &u, &v, &id)) return true;
            }
            h1 = false;
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
            if (sp == 0) return false;
            --sp;
            node = stack[sp * BLOCK];
        }
    }
}

// Pixel of lane `tid` in a 16 x 16 tile: each wave64 owns an 8 x 8 quadrant.
__device__ __forceinline__ void tile_pixel(int tid, int bx, int by, int* px, int* py)
{
    int w = tid >> 6, lane = tid & 63;
    *px = bx * 16 + (w & 1) * 8 + (lane & 7);
    *py = by * 16 + (w >> 1) * 8 + (lane >> 3);
}

template <bool COUNT>
__global__ __launch_bounds__(BLOCK) void k_gather(GatherArgs a)
{
    __shared__ float s_v[10][TILE_V];
    __shared__ int s_stack[kStack * BLOCK];
    const int tid = threadIdx.x;
    int px, py;
    tile_pixel(tid, blockIdx.x, blockIdx.y, &px, &py);
    const int W = a.gb.width, H = a.gb.height;
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
    const int M = *a.vpls.count;
    const float C = a.g_clamp;
    const float tlo = a.t_eps, thi = 1.0f - a.t_eps;
    int* stack = s_stack + tid;
    Counters cnt;
    unsigned long long pairs = 0;
    float ar = 0.f, ag = 0.f, ab = 0.f;
    for (int base = 0; base < M; base += TILE_V) {
        __syncthreads();
        int j = base + tid;
        if (j < M) {
            s_v[0][tid] = a.vpls.px[j]; s_v[1][tid] = a.vpls.py[j]; s_v[2][tid] = a.vpls.pz[j];
            s_v[3][tid] = a.vpls.nx[j]; s_v[4][tid] = a.vpls.ny[j]; s_v[5][tid] = a.vpls.nz[j];
            s_v[6][tid] = a.vpls.ir[j]; s_v[7][tid] = a.vpls.ig[j]; s_v[8][tid] = a.vpls.ib[j];
            s_v[9][tid] = __int_as_float(a.vpls.tri[j]);
        }
        __syncthreads();
        const int nt = min(TILE_V, M - base);
        float pr = 0.f, pg = 0.f, pb = 0.f;
        if (active) {
            if (COUNT) pairs += nt;
            for (int k = 0; k < nt; ++k) {
                float dx = s_v[0][k] - x, dy = s_v[1][k] - y, dz = s_v[2][k] - z;
                float cp = nx * dx + ny * dy + nz * dz;
                float ck = -(s_v[3][k] * dx + s_v[4][k] * dy + s_v[5][k] * dz);
                if (cp > 0.f && ck > 0.f) {
                    float r2 = dx * dx + dy * dy + dz * dz;
                    float g = fminf(C, cp * ck * rcpf(r2 * r2));
                    if (COUNT) cnt.rays++;
                    if (!occluded<COUNT>(a.scene, x, y, z, dx, dy, dz, tlo, thi, tp, __float_as_int(s_v[9][k]), stack,
                                         cnt)) {
                        pr = fmaf(s_v[6][k], g, pr);
                        pg = fmaf(s_v[7][k], g, pg);
                        pb = fmaf(s_v[8][k], g, pb);
                    }
                }
            }
        }
        ar += pr;
        ag += pg;
        ab += pb;
    }
    if (valid) {
        float s = kInvPi;
        a.out[0][p] = active ? a.gb.alb[0][p] * s * ar : 0.f;
        a.out[1][p] = active ? a.gb.alb[1][p] * s * ag : 0.f;
        a.out[2][p] = active ? a.gb.alb[2][p] * s * ab : 0.f;
    }
    if (COUNT) {
        unsigned long long v[4] = {pairs, cnt.rays, cnt.nodes, cnt.tris};
        for (int c = 0; c < 4; ++c) {
            unsigned long long s = v[c];
            for (int off = 32; off > 0; off >>= 1) s += __shfl_down(s, off, 64);
            if ((tid & 63) == 0) atomicAdd(&a.counters[c], s);
        }
    }
}

// One thread per (pixel, 32-VPL word): bit k of the word = V(x_p, y_k),
// evaluated for every pair with the gather's shadow-ray code.
__global__ __launch_bounds__(BLOCK) void k_vis_dump(VisDumpArgs a)
{
    __shared__ int s_stack[kStack * BLOCK];
    const int gid = blockIdx.x * BLOCK + threadIdx.x;
    const int total = a.n_px * a.words;
    if (gid >= total) return;
    const int i = gid / a.words, w = gid % a.words;
    const int p = a.pixels[i];
    const int M = *a.vpls.count;
    if (p < 0 || p >= a.gb.width * a.gb.height) {  // pixel list lives on the device: check it here
        a.bits[(size_t)i * a.words + w] = 0u;
        return;
    }
    const int tp = a.gb.tri[p];
    uint32_t bits = 0;
    Counters cnt;
    if (tp >= 0) {
        float x = a.gb.pos[0][p], y = a.gb.pos[1][p], z = a.gb.pos[2][p];
        for (int b = 0; b < 32; ++b) {
            int k = w * 32 + b;
            if (k >= M) break;
            float dx = a.vpls.px[k] - x, dy = a.vpls.py[k] - y, dz = a.vpls.pz[k] - z;
            bool occ = occluded<false>(a.scene, x, y, z, dx, dy, dz, a.t_eps, 1.0f - a.t_eps, tp, a.vpls.tri[k],
                                       s_stack + threadIdx.x, cnt);
            if (!occ) bits |= 1u << b;
        }
    }
    a.bits[(size_t)i * a.words + w] = bits;
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
    const float d2 = dx * dx + dy * dy + dz * dz;
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
        int k0 = __float_as_int(n3f.z), k1 = __float_as_int(n3f.w);
        float lo0, hi0, lo1, hi1;
        child_boxes(n0, n1, n2, r, 0.0f, best, &lo0, &hi0, &lo1, &hi1);
        bool h0 = lo0 <= hi0 && c0 >= 0;
        bool h1 = lo1 <= hi1 && c1 >= 0;
        for (int c = 0; c < 2; ++c) {
            bool h = c == 0 ? h0 : h1;
            int first = c == 0 ? c0 : c1, count = c == 0 ? k0 : k1;
            if (h && count > 0) {
                for (int i = first; i < first + count; ++i) {
                    float t, u, v;
                    int id;
                    bool ok = tri_hit32(tris, i, ox, oy, oz, dx, dy, dz, d2, 0.0f, __builtin_inff(), -2, -2, &t, &u,
                                        &v, &id);
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
    float4 v0 = tris[3 * bi], e1 = tris[3 * bi + 1], e2 = tris[3 * bi + 2];
    a.pos[0][p] = v0.x + bu * e1.x + bv * e2.x;
    a.pos[1][p] = v0.y + bu * e1.y + bv * e2.y;
    a.pos[2][p] = v0.z + bu * e1.z + bv * e2.z;
    float4 n = a.scene.normals[bid];
    a.nrm[0][p] = n.x; a.nrm[1][p] = n.y; a.nrm[2][p] = n.z;
    a.alb[0][p] = a.scene.albedo[3 * bid];
    a.alb[1][p] = a.scene.albedo[3 * bid + 1];
    a.alb[2][p] = a.scene.albedo[3 * bid + 2];
}

}  // namespace

hipError_t launch_gather(const GatherArgs& a, bool counted, hipStream_t s)
{
    dim3 grid((a.gb.width + 15) / 16, (a.gb.height + 15) / 16);
    if (counted)
        hipLaunchKernelGGL(k_gather<true>, grid, dim3(BLOCK), 0, s, a);
    else
        hipLaunchKernelGGL(k_gather<false>, grid, dim3(BLOCK), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_vis_dump(const VisDumpArgs& a, hipStream_t s)
{
    long long total = (long long)a.n_px * a.words;
    if (total == 0) return hipSuccess;
    dim3 grid((unsigned)((total + BLOCK - 1) / BLOCK));
    hipLaunchKernelGGL(k_vis_dump, grid, dim3(BLOCK), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_gbuffer(const GBufferArgs& a, hipStream_t s)
{
    dim3 grid((a.width + 15) / 16, (a.height + 15) / 16);
    hipLaunchKernelGGL(k_gbuffer, grid, dim3(BLOCK), 0, s, a);
    return hipGetLastError();
}

}  // namespace vplg
