// Internal declarations shared by the host runtime and the HIP kernels of the
// VPL library.  Not part of the ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace vplg {

// ---------------------------------------------------------------------------
// Device-resident scene
// ---------------------------------------------------------------------------
//
// BVH2 with both child boxes stored in the parent (one 64-byte node = four
// float4):
//   n0 = (c0.lo.x, c0.hi.x, c0.lo.y, c0.hi.y)
//   n1 = (c1.lo.x, c1.hi.x, c1.lo.y, c1.hi.y)
//   n2 = (c0.lo.z, c0.hi.z, c1.lo.z, c1.hi.z)
//   n3 = (int c0, int c1, int c0_count | c1_count << 16, int split)
// A child with count > 0 is a leaf holding triangles [c, c + count) of the
// leaf-ordered triangle array; count == 0 is an inner node.  Both children
// are always present (a scene that fits one leaf gets a root whose two
// children are that leaf).  split & 3 is the node's split axis, the axis
// along which the children's box centres lie farthest apart, child 0's the
// lower; split & ~3 is the position between the children along it,
// (c0.hi + c1.lo) / 2, as an order-preserving integer key of its float bits
// (b ^ ((b >> 31) & 0x7fffffff), two low bits dropped).  Node 0 is the root.
//
// Leaf-ordered triangles, four float4 each (one 64-byte scalar load):
// (A, id), (B, cut), (C, 0), (n, 0) with id = the original triangle index
// (bit pattern of an int), n = (B - A) x (C - A) and cut = (kParallelTau |n|)^2
// (+inf for a degenerate triangle, whose cut would round to zero).
// The FP32 ray tests are watertight (shared vertices are transformed
// identically for every triangle a ray tests, so a ray through a shared edge
// cannot slip between its two triangles) and treat a ray whose direction
// makes an angle below kParallelTau with the triangle's plane as missing it:
// there the projected triangle is degenerate at FP32 rounding, and any such
// ray that does cross the triangle is a grazing pair either answer serves.
constexpr double kParallelTau = 2e-5;
constexpr int kTriStride = 4;
constexpr int kMaxDepth = 48;   // builder guarantees depth <= kMaxDepth - 1
constexpr int kStack = 48;      // per-lane traversal stack entries

struct DevScene {
    int n_tris = 0;
    int n_nodes = 0;
    const float4* nodes = nullptr;    // 4 per node
    const float4* tris = nullptr;     // kTriStride per leaf-ordered triangle (identity order)
    // [3][n_tris] records: plane k has every vertex as (v[kx], v[ky], v[kz])
    // for dominant ray axis kz = k, kx and ky the next axes in cyclic order;
    // plane 2 is `tris`
    const float4* tris_rot = nullptr;
    const float* xyz = nullptr;       // original [T][3][3] float32
    const float* albedo = nullptr;    // [T][3]
    const uint8_t* flags = nullptr;   // [T]
    const float4* normals = nullptr;  // [T] unit face normal (float32 of the FP64 value)
    float lo[3], hi[3];               // scene bounding box (unpadded)
    double rho_bar = 0.0;             // mean albedo (area-weighted, non-emitting faces) for Keller's schedule
};

struct DevLight {
    int kind;  // 0 point, 1 quad
    float pos[3], eu[3], ev[3], power[3];
    // sample points of the light as eq. (2) uses them (computed in FP64 on the
    // host, stored as float32): the point itself, or the 16 quad cell centres
    // pos + eu (i + 1/2)/4 + ev (j + 1/2)/4 (sample j*4+i); nl = the quad's
    // unit normal edge_u x edge_v (its emitting side)
    int n_samples;
    float samples[16][3];
    float nl[3];
};

// VPL set in structure-of-arrays form; count on the device for generated sets.
struct DevVpls {
    float* px = nullptr; float* py = nullptr; float* pz = nullptr;
    float* nx = nullptr; float* ny = nullptr; float* nz = nullptr;
    float* ir = nullptr; float* ig = nullptr; float* ib = nullptr;
    int32_t* tri = nullptr;
    int32_t* count = nullptr;  // device int32: number of valid VPLs
    // gather layout: three float4 per VPL, (pos, tri bits), (nrm, free radius), (I, 0); the free radius
    // (the distance within which no triangle but the VPL's own and those in its plane lies) is that of
    // the scene the set was generated for, 0 for an uploaded set
    float4* pack = nullptr;
    int capacity = 0;
};

struct DevGBuffer {
    const float* pos[3];
    const float* nrm[3];
    const float* alb[3];
    const int32_t* tri;
    int width, height;
};

struct GatherArgs {
    DevScene scene;
    DevVpls vpls;
    DevGBuffer gb;
    float* out[3];
    float g_clamp;
    float t_eps;
    int waves_per_tile;            // VPL slices per 8 x 8 pixel tile: 1, 2, 4, 8 or 16
    // 8 x 8 tiles per work item (its pixel block): 1 (8 x 8), 2 (16 x 8) or
    // 4 (16 x 16); px_tiles * waves_per_tile <= 16.  A block's tiles are
    // gathered side by side, each by its own group of waves_per_tile waves,
    // so a pixel's sum depends on waves_per_tile only.
    int px_tiles;
    unsigned long long* counters;  // instrumented variant only
    // single-view gather only: split_part holds [split_cap][kGroups][3][64]
    // floats of work memory (split_cap 0: no tile is split); the launcher sets
    // split_full (whole blocks claimed first) and split_count (blocks after
    // it, claimed by round group; split_cap bounds split_count * px_tiles)
    int split_cap;
    int split_full, split_count;
    float* split_part;
    // which ends of the shadow segments are clipped by free radii: bit 0 the receivers' (walked per
    // tile), bit 1 the VPLs' (their records' radii, when the set was generated for this scene)
    int free_ends;
};

// Work table of a batched gather: views sorted by the caller, prefix[v] =
// first work item of view v (prefix[n_views] = total), waves[v] = waves per
// tile of view v (1, 2, 4, 8 or 16; the view's px_tiles is in its args).
constexpr int kBatchBlockWaves = 8;   // waves per persistent batch workgroup (views of <= 8 waves per tile)
constexpr int kBatchWideWaves = 16;   // the wide variant, used when a batch holds a 16-wave view
constexpr int kBatchMaxViews = 4096;
struct BatchTable {
    int n_views;
    int pad;
    int prefix[kBatchMaxViews + 1];
    int waves[kBatchMaxViews];
};

struct VisDumpArgs {
    DevScene scene;
    DevVpls vpls;
    DevGBuffer gb;
    const int32_t* pixels;
    int n_px;
    int words;  // ceil(capacity / 32)
    uint32_t* bits;
    float t_eps;
    int free_ends;  // as in GatherArgs
};

// Direct term L_e(y) of eq. (1) over a G-buffer.
struct DirectArgs {
    DevScene scene;
    DevLight light;
    DevGBuffer gb;
    float* out[3];
    float t_eps;
};

struct GBufferArgs {
    DevScene scene;
    float eye[3], f[3], r[3], u[3];
    float th, tx;
    float* pos[3];
    float* nrm[3];
    float* alb[3];
    int32_t* tri;
    int width, height;
};

// Camera basis in FP64 (host-computed, shared by the near test of generation).
struct CamBasis {
    double eye[3], f[3], r[3], u[3];
    double th, tx;  // tan(vfov / 2) and th * W / H
    int width, height;
};

struct GenParams {
    int k_near, n_far, max_bounces, max_paths;
    double d_near, patch_h, t_eps;
    int walk_near;   // 1: near hits after the first bounce become walk VPLs; 2: a near hit ends its path
    int jitter;      // 1: stratum targets jittered by the base-5 radical inverse of k + 1
    int brightness;  // 1: a patch VPL's flux is eq. (2) summed over its stratum's patches
    int walk_schedule;  // 1: Keller's schedule (N paths, path i goes on to bounce b iff i <= floor(rb^(b-1) N))
};

// Device-side record of one generation (counts are int64).
struct GenState {
    long long n_patches, n_near, n_eligible, q_total, k_eff, n_far_target, n_far, n_paths;
    long long far_b[3];
    long long flags, near_discarded;
    long long keller_n, keller_t[3];  // walk_schedule = 1: paths, and the path limit of each bounce
    int walk_done;
    int pad;
};

// Buffers of one generation.
struct GenBuffers {
    int n_patches;          // host-known total
    int32_t* level;         // [T] refinement level of each triangle
    long long* patch_off;   // [T + 1]
    uint8_t* pflags;        // [n_patches]
    unsigned long long* sortbuf;  // [pow2 >= n_patches] (key << 32 | patch): eligible patches first, then all-ones
    double* patch_g;        // = sortbuf once the order is extracted: eq. (2)'s light factor per sorted patch
    int32_t* sorted;        // [n_patches]
    uint32_t* keys;         // [n_patches]
    long long* F;           // [n_patches]
    int32_t* strata;        // [k_near]
    int32_t* vpl_path;      // [capacity]
    int32_t* vpl_bounce;    // [capacity]
    GenState* state;        // device
    long long* q;           // [n_patches] fixed-point areas in sorted order
    long long* scan_out;    // [n_patches + 1] exclusive prefix of q (F = scan_out + 1)
    double* stage_pos;      // [capacity][3] VPL positions before rounding to float
    double* stage_flux;     // [capacity][3] walk fluxes before normalisation
    // walk scratch for one batch of paths
    int batch;              // capacity in paths
    int32_t* w_count;       // [batch] far deposits | discard mask << 8
    double* w_pos;          // [batch][3][3]
    double* w_flux;         // [batch][3][3]
    int32_t* w_tri;         // [batch][3]
    int32_t* w_bounce;      // [batch][3]
    long long* scan_tmp;    // scan scratch
    int scan_tmp_len;
};

// ---------------------------------------------------------------------------
// Launchers (defined in the .hip files)
// ---------------------------------------------------------------------------
// Scenes of fewer triangles gather without free radii: their walks are short,
// and the receivers' radius walks would cost more than the clipping saves.
constexpr int kFreeMinTris = 1024;

// Persistent single-view gather: resets `counter` (a device word private to
// stream `s`) and launches `blocks` workgroups that claim tiles from it.
hipError_t launch_gather(const GatherArgs& a, bool counted, unsigned int* counter, int blocks, hipStream_t s);
// Resident workgroups per CU of the single-view gather for workgroups of `waves` waves.
hipError_t gather_occupancy(int waves, bool counted, int* blocks_per_cu);
// Pixel blocks of px_tiles 8 x 8 tiles (1, 2 or 4) covering a view.
int gather_view_blocks(int width, int height, int px_tiles);
// Floats of split-tile work memory per tile (its round groups' sums).
int gather_split_floats_per_tile();
// Allocation-free gather: its work memory is a fixed device array of the
// library (one per device).  Setup looks up the array's device address on the
// current device (once per device; call with `device` current); the address
// is then what the launches take.  Until setup has run on a device its
// address is null.
hipError_t gather_scratch_setup(int device);
void* gather_scratch_address(int device);
size_t gather_scratch_bytes();
int gather_scratch_split_cap();
// The persistent single-view gather with its tile counter and split-tile sums
// in `scratch` (an address from gather_scratch_address).
hipError_t launch_gather_scratch(const GatherArgs& a, void* scratch, int blocks, hipStream_t s);
hipError_t launch_vis_dump(const VisDumpArgs& a, hipStream_t s);
hipError_t launch_gather_batch(const BatchTable* tab, const GatherArgs* views, unsigned int* counter, int blocks,
                               int block_waves, hipStream_t s);
hipError_t gather_batch_occupancy(int block_waves, int* blocks_per_cu);
hipError_t launch_gbuffer(const GBufferArgs& a, hipStream_t s);
hipError_t launch_direct(const DirectArgs& a, hipStream_t s);
// Pack the gather's VPL records; with a scene (non-null), each VPL's free radius in it.
hipError_t launch_pack_vpls(const DevScene* sc, const DevVpls& v, hipStream_t s);

hipError_t launch_patch_levels(const DevScene& sc, double h, int32_t* level, long long* counts, hipStream_t s);
hipError_t launch_scan_i64(const long long* in, long long* out, int n, long long* tmp, int tmp_len,
                           hipStream_t s);  // exclusive scan, out[n] = total
int scan_tmp_needed(int n);
hipError_t launch_generate(const DevScene& sc, const DevLight& L, const CamBasis& cam, const GenParams& p,
                           const DevVpls& v, const GenBuffers& b, hipStream_t s);

}  // namespace vplg
