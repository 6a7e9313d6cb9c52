// Internal state of the host runtime, shared by runtime.cpp and server.cpp.
// Not part of the ABI.
#pragma once

#include <cstdarg>
#include <deque>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "vplg.h"
#include "vplg_impl.h"

namespace vplg {

bool build_bvh(const float* xyz, int T, std::vector<float4>& out_nodes, std::vector<float4>& out_tris, int* n_leaves,
               int* max_depth, std::string& err);

namespace rt {

extern thread_local std::string g_err;
int fail(int code, const char* fmt, ...);

#define HIPCHK(expr)                                                                                   \
    do {                                                                                               \
        hipError_t e_ = (expr);                                                                        \
        if (e_ != hipSuccess) return ::vplg::rt::fail(VPLG_EHIP, "%s: %s", #expr, hipGetErrorString(e_)); \
    } while (0)

struct Alloc {
    void* p;
    size_t bytes;
};

struct PatchIndex {
    double h;
    int32_t* level;
    long long* off;
    long long total;
};

struct SceneObj {
    uint64_t id = 0;
    DevScene dev;
    DevLight light;
    std::vector<Alloc> allocs;
    uint64_t bytes = 0;
    vplg_scene_info info;
    // one index per patch size; a deque, so that the index a caller holds
    // stays in place when another thread adds one for another size
    std::deque<PatchIndex> patches;
};

struct VplSetObj {
    DevVpls dev;
    std::vector<Alloc> allocs;
    uint64_t bytes = 0;
    bool generated = false;
    GenBuffers gen;
    int k_near = 0;
    int n_far = 0;
    int n_tris = 0;
    uint64_t scene_id = 0;
    double patch_h = 0.0;
    hipEvent_t done = nullptr;
    // the scene whose free radii the VPL records hold (0: none, an uploaded set)
    uint64_t radius_scene = 0;
};

// Persistent batched gather: device work table and view descriptors, their
// pinned staging, and the HIP graph of (counter reset + persistent kernel).
struct BatchEngine {
    BatchTable* d_tab = nullptr;
    GatherArgs* d_views = nullptr;
    unsigned int* d_counter = nullptr;
    BatchTable* h_tab = nullptr;
    GatherArgs* h_views = nullptr;
    hipEvent_t staged = nullptr;  // last use of the pinned staging
    hipEvent_t replayed = nullptr;  // end of the last replay (the device table's last reader)
    hipStream_t capture = nullptr;
    // [0]: workgroups of 8 waves, [1]: of 16 waves (captured on first use)
    hipGraph_t graph[2] = {nullptr, nullptr};
    hipGraphExec_t exec[2] = {nullptr, nullptr};
    int blocks[2] = {0, 0};
    bool ready = false;
};

}  // namespace rt
}  // namespace vplg

namespace vplg {
namespace rt {
// Per-stream work memory of the single-view gather: its tile counter and the
// round-group sums of up to kGatherSplitCap split tiles.
constexpr int kGatherSplitCap = 2048;
// waves of a single-view gather workgroup at most (tiles per block x waves per tile)
constexpr int kGatherMaxWorkgroupWaves = 16;
struct GatherWork {
    unsigned int* counter = nullptr;
    float* part = nullptr;
};
// Tile shape of a gather: waves per 8 x 8 tile (the VPL slices whose partial
// sums fix a pixel's summation order) and 8 x 8 tiles per work item (its
// pixel block: 1, 2 or 4, gathered side by side in one workgroup).
struct TileShape {
    int waves = 8, px_tiles = 1;
};
}  // namespace rt
}  // namespace vplg

struct vplg_context {
    int device = 0;
    uint64_t budget = 0, used = 0;
    uint64_t next_id = 1;
    std::map<uint64_t, vplg::rt::SceneObj*> scenes;
    std::map<uint64_t, vplg::rt::VplSetObj*> sets;
    vplg::rt::BatchEngine batch;
    // view-shape bucket -> tuned tile shape, for lone gathers and for views
    // inside a batch (tuned with the batched launch as the objective)
    std::map<uint32_t, vplg::rt::TileShape> tuned, tuned_batch;
    // work memory of the persistent single-view gather, per stream (launches
    // on one stream are ordered, so they may share it)
    std::map<void*, vplg::rt::GatherWork> stream_work;
    int cus = 0;                      // compute units of the device
    int gather_blocks[2][5] = {};     // [counted][log2 workgroup waves]: resident workgroups per CU, 0 = not queried
    std::recursive_mutex mu;        // budget accounting, shared with a running server thread
};

namespace vplg {
namespace rt {

int dalloc(vplg_context* ctx, std::vector<Alloc>& list, uint64_t& acc, size_t bytes, void** out);
template <class T>
int dalloc_n(vplg_context* ctx, std::vector<Alloc>& list, uint64_t& acc, size_t n, T** out)
{
    void* p = nullptr;
    int rc = dalloc(ctx, list, acc, n * sizeof(T), &p);
    *out = (T*)p;
    return rc;
}
void free_all(vplg_context* ctx, std::vector<Alloc>& list);
int set_device(vplg_context* ctx);
SceneObj* find_scene(vplg_context* ctx, uint64_t id);
VplSetObj* find_set(vplg_context* ctx, uint64_t id);
void release_set(vplg_context* ctx, VplSetObj* v);
CamBasis cam_basis(const vplg_camera* c);
int check_camera(const vplg_camera* c);
int check_gbuffer(const vplg_gbuffer* gb);
int check_gen_params(const vplg_gen_params* p);
DevGBuffer dev_gbuffer(const vplg_gbuffer* gb);
int wait_set(VplSetObj* v);
int set_count(VplSetObj* v, int32_t* n);
// G-buffer kernel of a resident scene (arguments already checked)
int render_gbuffer(SceneObj* so, const vplg_camera* cam, const vplg_gbuffer* gb, hipStream_t s);
// patch index of a scene for patch_h (first use synchronises `s`)
int patch_index(vplg_context* ctx, SceneObj* so, double h, hipStream_t s, PatchIndex** out);
// device bytes a generated set of this shape holds
uint64_t genset_bytes(long long n_patches, int k_near, int n_far);
// allocate a generated set (no launch); launch (or relaunch) its generation
int alloc_genset(vplg_context* ctx, SceneObj* so, uint64_t scene_id, PatchIndex* pi, const vplg_gen_params* p,
                 VplSetObj** out);
int launch_genset(SceneObj* so, VplSetObj* v, const vplg_camera* cam, const vplg_gen_params* p, hipStream_t s);
constexpr int kWideTilesPerCu = 32;
// view-shape bucket of the autotuner: ceil(log2(pixels)) << 8 | ceil(log2(VPLs))
uint32_t shape_bucket(int width, int height, int n_vpls);
// tile shape of a view whose parameters leave it open (tile_vpl 0): the
// autotuned choice for its shape (lone or batched table), else 8 x 8 pixel
// blocks with, for a view launched alone, 16 waves per tile when it has fewer
// than kWideTilesPerCu tiles per CU (shorter work items shorten the launch's
// tail) and 8 above; a view in a batch gets 8 (the batch shares one tail, and
// 16-wave workgroups would tie the 8-wave views' tile pairs to common barriers)
TileShape tuned_shape(vplg_context* ctx, int width, int height, int n_vpls, bool batched);
int gather_common(vplg_context* ctx, uint64_t scene_id, uint64_t vplset_id, const vplg_gbuffer* gb,
                  float* const radiance[3], const vplg_gather_params* p, GatherArgs* a, bool batched = false);
int gather_args(vplg_context* ctx, SceneObj* so, VplSetObj* v, const vplg_gbuffer* gb, float* const radiance[3],
                const vplg_gather_params* p, GatherArgs* a, bool batched = false);
// launch the persistent single-view gather of `a` on `s` (its stream's tile counter, resident grid)
// split_tail = false: whole tiles only (for gathers that share the GPU with
// others, where no one view's tail leaves it idle); the result is the same.
int run_gather(vplg_context* ctx, const GatherArgs& a, bool counted, hipStream_t s, bool split_tail = true);
// resident workgroups of the single-view gather for workgroups of `waves` waves (cached per context)
int gather_grid(vplg_context* ctx, int waves, bool counted, int* blocks);

}  // namespace rt
}  // namespace vplg
