// Host runtime behind include/vplg.h: contexts with an HBM budget, resident
// scenes (host SAH BVH) and VPL sets, argument checking, and the dispatch of
// the G-buffer, generation and gather kernels.
#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <string>
#include <vector>


#include "runtime_internal.h"

using namespace vplg;
using namespace vplg::rt;

namespace vplg {
namespace rt {

thread_local std::string g_err;

int fail(int code, const char* fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

int dalloc(vplg_context* ctx, std::vector<Alloc>& list, uint64_t& acc, size_t bytes, void** out)
{
    std::lock_guard<std::recursive_mutex> lock(ctx->mu);
    if (bytes == 0) bytes = 16;
    bytes = (bytes + 255) & ~(size_t)255;
    if (ctx->budget && ctx->used + bytes > ctx->budget)
        return fail(VPLG_EBUDGET, "HBM budget exceeded: %llu used + %llu requested > %llu",
                    (unsigned long long)ctx->used, (unsigned long long)bytes, (unsigned long long)ctx->budget);
    void* p = nullptr;
    hipError_t e = hipMalloc(&p, bytes);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return fail(VPLG_ENOMEM, "hipMalloc(%llu) failed: %s", (unsigned long long)bytes, hipGetErrorString(e));
    }
    list.push_back({p, bytes});
    acc += bytes;
    ctx->used += bytes;
    *out = p;
    return VPLG_OK;
}

void free_all(vplg_context* ctx, std::vector<Alloc>& list)
{
    std::lock_guard<std::recursive_mutex> lock(ctx->mu);
    for (auto& a : list) {
        (void)hipFree(a.p);
        ctx->used -= a.bytes;
    }
    list.clear();
}

int set_device(vplg_context* ctx)
{
    if (!ctx) return fail(VPLG_EINVAL, "null context");
    HIPCHK(hipSetDevice(ctx->device));
    return VPLG_OK;
}

SceneObj* find_scene(vplg_context* ctx, uint64_t id)
{
    std::lock_guard<std::recursive_mutex> lock(ctx->mu);
    auto it = ctx->scenes.find(id);
    return it == ctx->scenes.end() ? nullptr : it->second;
}

VplSetObj* find_set(vplg_context* ctx, uint64_t id)
{
    std::lock_guard<std::recursive_mutex> lock(ctx->mu);
    auto it = ctx->sets.find(id);
    return it == ctx->sets.end() ? nullptr : it->second;
}

void release_set(vplg_context* ctx, VplSetObj* v)
{
    if (v->done) (void)hipEventDestroy(v->done);
    free_all(ctx, v->allocs);
    delete v;
}

// Camera basis in FP64: f = normalize(target - eye), r = normalize(f x up),
// u = r x f, th = tan(vfov / 2), tx = th W / H (fixed operation order).
CamBasis cam_basis(const vplg_camera* c)
{
    CamBasis k;
    double eye[3], tg[3], up[3];
    for (int i = 0; i < 3; ++i) {
        eye[i] = c->eye[i];
        tg[i] = c->target[i];
        up[i] = c->up[i];
    }
    double f[3] = {tg[0] - eye[0], tg[1] - eye[1], tg[2] - eye[2]};
    double lf = std::sqrt(f[0] * f[0] + f[1] * f[1] + f[2] * f[2]);
    for (int i = 0; i < 3; ++i) f[i] = f[i] / lf;
    double r[3] = {f[1] * up[2] - f[2] * up[1], f[2] * up[0] - f[0] * up[2], f[0] * up[1] - f[1] * up[0]};
    double lr = std::sqrt(r[0] * r[0] + r[1] * r[1] + r[2] * r[2]);
    for (int i = 0; i < 3; ++i) r[i] = r[i] / lr;
    double u[3] = {r[1] * f[2] - r[2] * f[1], r[2] * f[0] - r[0] * f[2], r[0] * f[1] - r[1] * f[0]};
    for (int i = 0; i < 3; ++i) {
        k.eye[i] = eye[i];
        k.f[i] = f[i];
        k.r[i] = r[i];
        k.u[i] = u[i];
    }
    k.width = c->width;
    k.height = c->height;
    k.th = std::tan((double)c->vfov_deg * (3.14159265358979323846 / 360.0));
    k.tx = k.th * ((double)c->width / (double)c->height);
    return k;
}

int check_camera(const vplg_camera* c)
{
    if (!c) return fail(VPLG_EINVAL, "null camera");
    if (c->width < 1 || c->height < 1 || (long long)c->width * c->height > (1ll << 28))
        return fail(VPLG_EINVAL, "bad image size %d x %d", c->width, c->height);
    if (!(c->vfov_deg > 0.f && c->vfov_deg < 180.f)) return fail(VPLG_EINVAL, "vfov must be in (0, 180)");
    double f[3] = {(double)c->target[0] - c->eye[0], (double)c->target[1] - c->eye[1],
                   (double)c->target[2] - c->eye[2]};
    double cr[3] = {f[1] * c->up[2] - f[2] * c->up[1], f[2] * c->up[0] - f[0] * c->up[2],
                    f[0] * c->up[1] - f[1] * c->up[0]};
    if (f[0] * f[0] + f[1] * f[1] + f[2] * f[2] == 0.0 || cr[0] * cr[0] + cr[1] * cr[1] + cr[2] * cr[2] == 0.0)
        return fail(VPLG_EINVAL, "degenerate camera basis");
    return VPLG_OK;
}

int check_gbuffer(const vplg_gbuffer* gb)
{
    if (!gb) return fail(VPLG_EINVAL, "null gbuffer");
    for (int c = 0; c < 3; ++c)
        if (!gb->pos[c] || !gb->nrm[c] || !gb->alb[c]) return fail(VPLG_EINVAL, "null gbuffer plane");
    if (!gb->tri) return fail(VPLG_EINVAL, "null gbuffer tri plane");
    if (gb->width < 1 || gb->height < 1 || (long long)gb->width * gb->height > (1ll << 28))
        return fail(VPLG_EINVAL, "bad gbuffer size %d x %d", gb->width, gb->height);
    return VPLG_OK;
}

DevGBuffer dev_gbuffer(const vplg_gbuffer* gb)
{
    DevGBuffer d;
    for (int c = 0; c < 3; ++c) {
        d.pos[c] = gb->pos[c];
        d.nrm[c] = gb->nrm[c];
        d.alb[c] = gb->alb[c];
    }
    d.tri = gb->tri;
    d.width = gb->width;
    d.height = gb->height;
    return d;
}

int wait_set(VplSetObj* v)
{
    if (v->done) HIPCHK(hipEventSynchronize(v->done));
    return VPLG_OK;
}

int set_count(VplSetObj* v, int32_t* n)
{
    int rc = wait_set(v);
    if (rc) return rc;
    HIPCHK(hipMemcpy(n, v->dev.count, sizeof(int32_t), hipMemcpyDeviceToHost));
    return VPLG_OK;
}

}  // namespace rt
}  // namespace vplg

extern "C" {

const char* vplg_last_error(void) { return g_err.c_str(); }

int vplg_version(void) { return 10000; }

int vplg_context_create(int device, uint64_t hbm_budget_bytes, vplg_context** out)
{
    if (!out) return fail(VPLG_EINVAL, "null output pointer");
    *out = nullptr;
    int n = 0;
    HIPCHK(hipGetDeviceCount(&n));
    if (device < 0 || device >= n) return fail(VPLG_EINVAL, "device %d out of range (%d devices)", device, n);
    HIPCHK(hipSetDevice(device));
    // the allocation-free gather's work memory: its address on this device
    hipError_t e = gather_scratch_setup(device);
    if (e != hipSuccess) return fail(VPLG_EHIP, "gather scratch address on device %d: %s", device, hipGetErrorString(e));
    auto* ctx = new vplg_context;
    ctx->device = device;
    ctx->budget = hbm_budget_bytes;
    *out = ctx;
    return VPLG_OK;
}

int vplg_context_destroy(vplg_context* ctx)
{
    if (!ctx) return fail(VPLG_EINVAL, "null context");
    (void)hipSetDevice(ctx->device);
    (void)hipDeviceSynchronize();
    for (auto& kv : ctx->sets) release_set(ctx, kv.second);
    for (auto& kv : ctx->scenes) {
        free_all(ctx, kv.second->allocs);
        delete kv.second;
    }
    BatchEngine& be = ctx->batch;
    for (int i = 0; i < 2; ++i) {
        if (be.exec[i]) (void)hipGraphExecDestroy(be.exec[i]);
        if (be.graph[i]) (void)hipGraphDestroy(be.graph[i]);
    }
    if (be.capture) (void)hipStreamDestroy(be.capture);
    if (be.staged) (void)hipEventDestroy(be.staged);
    if (be.replayed) (void)hipEventDestroy(be.replayed);
    if (be.d_tab) (void)hipFree(be.d_tab);
    if (be.d_views) (void)hipFree(be.d_views);
    if (be.d_counter) (void)hipFree(be.d_counter);
    if (be.h_tab) (void)hipHostFree(be.h_tab);
    if (be.h_views) (void)hipHostFree(be.h_views);
    for (auto& kv : ctx->stream_work) {
        (void)hipFree(kv.second.counter);
        (void)hipFree(kv.second.part);
    }
    delete ctx;
    return VPLG_OK;
}

int vplg_context_usage(vplg_context* ctx, uint64_t* used, uint64_t* budget)
{
    if (!ctx) return fail(VPLG_EINVAL, "null context");
    std::lock_guard<std::recursive_mutex> lock(ctx->mu);
    if (used) *used = ctx->used;
    if (budget) *budget = ctx->budget;
    return VPLG_OK;
}

// Mean albedo of Keller's path schedule: face-area-weighted over the faces
// that do not emit, of the mean of the three channels (0 without such area).
// FP64 in triangle order; built without contraction.
static double mean_albedo(const float* xyz, const float* alb, const uint8_t* flags, int T)
{
    double num = 0.0, den = 0.0;
    for (int t = 0; t < T; ++t) {
        if (flags[t] & 1) continue;
        const float* p = xyz + 9 * (size_t)t;
        const double e1[3] = {(double)p[3] - (double)p[0], (double)p[4] - (double)p[1], (double)p[5] - (double)p[2]};
        const double e2[3] = {(double)p[6] - (double)p[0], (double)p[7] - (double)p[1], (double)p[8] - (double)p[2]};
        const double cr[3] = {e1[1] * e2[2] - e1[2] * e2[1], e1[2] * e2[0] - e1[0] * e2[2],
                              e1[0] * e2[1] - e1[1] * e2[0]};
        const double a = 0.5 * std::sqrt(cr[0] * cr[0] + cr[1] * cr[1] + cr[2] * cr[2]);
        const double m = (((double)alb[3 * t] + (double)alb[3 * t + 1]) + (double)alb[3 * t + 2]) / 3.0;
        num += a * m;
        den += a;
    }
    return den > 0.0 ? num / den : 0.0;
}

int vplg_scene_upload(vplg_context* ctx, const float* tri_xyz, const float* tri_albedo, const uint8_t* tri_flags,
                      int32_t n_tris, const vplg_light* light, void* stream, uint64_t* scene_id)
{
    int rc = set_device(ctx);
    if (rc) return rc;
    if (!tri_xyz || !tri_albedo || !tri_flags || !light || !scene_id) return fail(VPLG_EINVAL, "null argument");
    // at most 2^25 triangles: node and triangle records (64 bytes each, fewer
    // than 2 n_tris nodes) are then addressed by 32-bit byte offsets
    if (n_tris < 1 || n_tris > (1 << 25)) return fail(VPLG_EINVAL, "n_tris %d out of range", n_tris);
    if (light->kind != 0 && light->kind != 1) return fail(VPLG_EINVAL, "unknown light kind %d", light->kind);
    for (size_t i = 0; i < 9 * (size_t)n_tris; ++i)
        if (!std::isfinite(tri_xyz[i])) return fail(VPLG_EINVAL, "non-finite vertex coordinate at %zu", i);
    hipStream_t s = (hipStream_t)stream;
    std::vector<float4> nodes, tris;
    int n_leaves = 0, depth = 0;
    std::string err;
    if (!build_bvh(tri_xyz, n_tris, nodes, tris, &n_leaves, &depth, err)) return fail(VPLG_EINVAL, "%s", err.c_str());
    std::vector<float4> normals(n_tris);
    SceneObj* so = new SceneObj;
    DevScene& d = so->dev;
    for (int k = 0; k < 3; ++k) {
        d.lo[k] = tri_xyz[k];
        d.hi[k] = tri_xyz[k];
    }
    for (int t = 0; t < n_tris; ++t) {
        const float* p = tri_xyz + 9 * (size_t)t;
        double a[3], b[3], c[3];
        for (int k = 0; k < 3; ++k) {
            a[k] = p[k];
            b[k] = p[3 + k];
            c[k] = p[6 + k];
            for (int v = 0; v < 3; ++v) {
                d.lo[k] = std::min(d.lo[k], p[3 * v + k]);
                d.hi[k] = std::max(d.hi[k], p[3 * v + k]);
            }
        }
        double e1[3] = {b[0] - a[0], b[1] - a[1], b[2] - a[2]};
        double e2[3] = {c[0] - a[0], c[1] - a[1], c[2] - a[2]};
        double n[3] = {e1[1] * e2[2] - e1[2] * e2[1], e1[2] * e2[0] - e1[0] * e2[2], e1[0] * e2[1] - e1[1] * e2[0]};
        double l = std::sqrt(n[0] * n[0] + n[1] * n[1] + n[2] * n[2]);
        if (l > 0) normals[t] = make_float4((float)(n[0] / l), (float)(n[1] / l), (float)(n[2] / l), 0.f);
        else normals[t] = make_float4(0.f, 0.f, 0.f, 0.f);
    }
    float4 *dn = nullptr, *dt = nullptr, *dnorm = nullptr;
    float *dxyz = nullptr, *dalb = nullptr;
    uint8_t* dfl = nullptr;
    if ((rc = dalloc_n(ctx, so->allocs, so->bytes, nodes.size(), &dn)) ||
        (rc = dalloc_n(ctx, so->allocs, so->bytes, tris.size(), &dt)) ||
        (rc = dalloc_n(ctx, so->allocs, so->bytes, 9 * (size_t)n_tris, &dxyz)) ||
        (rc = dalloc_n(ctx, so->allocs, so->bytes, 3 * (size_t)n_tris, &dalb)) ||
        (rc = dalloc_n(ctx, so->allocs, so->bytes, (size_t)n_tris, &dfl)) ||
        (rc = dalloc_n(ctx, so->allocs, so->bytes, (size_t)n_tris, &dnorm))) {
        free_all(ctx, so->allocs);
        delete so;
        return rc;
    }
    hipError_t e = hipSuccess;
    if (e == hipSuccess) e = hipMemcpyAsync(dn, nodes.data(), nodes.size() * sizeof(float4), hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipMemcpyAsync(dt, tris.data(), tris.size() * sizeof(float4), hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipMemcpyAsync(dxyz, tri_xyz, 36 * (size_t)n_tris, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipMemcpyAsync(dalb, tri_albedo, 12 * (size_t)n_tris, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipMemcpyAsync(dfl, tri_flags, (size_t)n_tris, hipMemcpyHostToDevice, s);
    if (e == hipSuccess)
        e = hipMemcpyAsync(dnorm, normals.data(), normals.size() * sizeof(float4), hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) {
        free_all(ctx, so->allocs);
        delete so;
        return fail(VPLG_EHIP, "scene upload copy failed: %s", hipGetErrorString(e));
    }
    d.n_tris = n_tris;
    d.n_nodes = (int)(nodes.size() / 4);
    d.nodes = dn;
    d.tris_rot = dt;
    d.tris = dt + 2 * kTriStride * (size_t)n_tris;
    d.xyz = dxyz;
    d.albedo = dalb;
    d.flags = dfl;
    d.normals = dnorm;
    d.rho_bar = mean_albedo(tri_xyz, tri_albedo, tri_flags, n_tris);
    so->light.kind = light->kind;
    for (int k = 0; k < 3; ++k) {
        so->light.pos[k] = light->pos[k];
        so->light.eu[k] = light->edge_u[k];
        so->light.ev[k] = light->edge_v[k];
        so->light.power[k] = light->power[k];
    }
    // the light's sample points in FP64 (the point, or the 16 cell centres)
    {
        const double P[3] = {light->pos[0], light->pos[1], light->pos[2]};
        const double U[3] = {light->edge_u[0], light->edge_u[1], light->edge_u[2]};
        const double V[3] = {light->edge_v[0], light->edge_v[1], light->edge_v[2]};
        so->light.n_samples = light->kind == 0 ? 1 : 16;
        for (int j = 0; j < so->light.n_samples; ++j) {
            const double a = light->kind == 0 ? 0.0 : ((double)(j % 4) + 0.5) / 4.0;
            const double b = light->kind == 0 ? 0.0 : ((double)(j / 4) + 0.5) / 4.0;
            for (int k = 0; k < 3; ++k) so->light.samples[j][k] = (float)((P[k] + U[k] * a) + V[k] * b);
        }
        const double n[3] = {U[1] * V[2] - U[2] * V[1], U[2] * V[0] - U[0] * V[2], U[0] * V[1] - U[1] * V[0]};
        const double l = std::sqrt(n[0] * n[0] + n[1] * n[1] + n[2] * n[2]);
        for (int k = 0; k < 3; ++k) so->light.nl[k] = l > 0 ? (float)(n[k] / l) : 0.f;
    }
    so->info.n_tris = n_tris;
    so->info.n_nodes = d.n_nodes;
    so->info.n_leaves = n_leaves;
    so->info.max_depth = depth;
    so->info.device_bytes = so->bytes;
    for (int k = 0; k < 3; ++k) {
        so->info.lo[k] = d.lo[k];
        so->info.hi[k] = d.hi[k];
    }
    std::lock_guard<std::recursive_mutex> lock(ctx->mu);
    uint64_t id = ctx->next_id++;
    so->id = id;
    ctx->scenes[id] = so;
    *scene_id = id;
    return VPLG_OK;
}

int vplg_scene_release(vplg_context* ctx, uint64_t scene_id)
{
    int rc = set_device(ctx);
    if (rc) return rc;
    SceneObj* so = find_scene(ctx, scene_id);
    if (!so) return fail(VPLG_ENOTFOUND, "unknown scene %llu", (unsigned long long)scene_id);
    HIPCHK(hipDeviceSynchronize());
    std::lock_guard<std::recursive_mutex> lock(ctx->mu);
    free_all(ctx, so->allocs);
    delete so;
    ctx->scenes.erase(scene_id);
    return VPLG_OK;
}

int vplg_scene_describe(vplg_context* ctx, uint64_t scene_id, vplg_scene_info* out)
{
    if (!ctx || !out) return fail(VPLG_EINVAL, "null argument");
    SceneObj* so = find_scene(ctx, scene_id);
    if (!so) return fail(VPLG_ENOTFOUND, "unknown scene %llu", (unsigned long long)scene_id);
    *out = so->info;
    out->device_bytes = so->bytes;
    return VPLG_OK;
}

}  // extern "C"

namespace vplg {
namespace rt {

int render_gbuffer(SceneObj* so, const vplg_camera* cam, const vplg_gbuffer* gb, hipStream_t s)
{
    CamBasis k = cam_basis(cam);
    GBufferArgs a;
    a.scene = so->dev;
    for (int i = 0; i < 3; ++i) {
        a.eye[i] = (float)k.eye[i];
        a.f[i] = (float)k.f[i];
        a.r[i] = (float)k.r[i];
        a.u[i] = (float)k.u[i];
        a.pos[i] = gb->pos[i];
        a.nrm[i] = gb->nrm[i];
        a.alb[i] = gb->alb[i];
    }
    a.th = (float)k.th;
    a.tx = (float)k.tx;
    a.tri = gb->tri;
    a.width = gb->width;
    a.height = gb->height;
    HIPCHK(launch_gbuffer(a, s));
    return VPLG_OK;
}

int check_gen_params(const vplg_gen_params* p)
{
    if (!p) return fail(VPLG_EINVAL, "null parameters");
    if (p->k_near < 0 || p->n_far < 0 || (long long)p->k_near + p->n_far > (1 << 26))
        return fail(VPLG_EINVAL, "bad VPL budget k_near=%d n_far=%d", p->k_near, p->n_far);
    if (p->max_bounces < 1 || p->max_bounces > 3) return fail(VPLG_EINVAL, "max_bounces must be in [1, 3]");
    if (p->max_paths < 1) return fail(VPLG_EINVAL, "max_paths must be >= 1");
    if (!(p->patch_h > 0.0) || !std::isfinite(p->patch_h)) return fail(VPLG_EINVAL, "patch_h must be > 0");
    if (!(p->d_near >= 0.0)) return fail(VPLG_EINVAL, "d_near must be >= 0");
    if (!(p->t_eps >= 0.0 && p->t_eps < 0.5)) return fail(VPLG_EINVAL, "t_eps must be in [0, 0.5)");
    if (p->walk_near < 0 || p->walk_near > 2) return fail(VPLG_EINVAL, "walk_near must be 0, 1 or 2");
    if (p->jitter != 0 && p->jitter != 1) return fail(VPLG_EINVAL, "jitter must be 0 or 1");
    if (p->brightness != 0 && p->brightness != 1) return fail(VPLG_EINVAL, "brightness must be 0 or 1");
    if (p->walk_schedule != 0 && p->walk_schedule != 1) return fail(VPLG_EINVAL, "walk_schedule must be 0 or 1");
    return VPLG_OK;
}

int patch_index(vplg_context* ctx, SceneObj* so, double h, hipStream_t s, PatchIndex** out)
{
    std::lock_guard<std::recursive_mutex> lock(ctx->mu);
    for (auto& x : so->patches)
        if (x.h == h) {
            *out = &x;
            return VPLG_OK;
        }
    const int T = so->dev.n_tris;
    PatchIndex x;
    x.h = h;
    long long* counts = nullptr;
    std::vector<Alloc> tmp;
    uint64_t tmp_bytes = 0;
    long long* scan_tmp = nullptr;
    int need = scan_tmp_needed(T);
    int rc;
    if ((rc = dalloc_n(ctx, so->allocs, so->bytes, (size_t)T, &x.level)) ||
        (rc = dalloc_n(ctx, so->allocs, so->bytes, (size_t)T + 1, &x.off)) ||
        (rc = dalloc_n(ctx, tmp, tmp_bytes, (size_t)T, &counts)) ||
        (rc = dalloc_n(ctx, tmp, tmp_bytes, (size_t)need, &scan_tmp))) {
        free_all(ctx, tmp);
        return rc;
    }
    hipError_t e = launch_patch_levels(so->dev, h, x.level, counts, s);
    if (e == hipSuccess) e = launch_scan_i64(counts, x.off, T, scan_tmp, need, s);
    if (e == hipSuccess) e = hipMemcpyAsync(&x.total, x.off + T, sizeof(long long), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    free_all(ctx, tmp);
    if (e != hipSuccess) return fail(VPLG_EHIP, "patch index: %s", hipGetErrorString(e));
    if (x.total > (1ll << 30)) return fail(VPLG_EINVAL, "too many patches (%lld) for patch_h", x.total);
    so->patches.push_back(x);
    so->info.device_bytes = so->bytes;
    *out = &so->patches.back();
    return VPLG_OK;
}

namespace {

// Allocation plan of a generated set: element counts of every array.
struct GensetShape {
    size_t cap1, np1, n2, strata;
    int batch, scan_tmp_len;
};

GensetShape genset_shape(long long NP, int k_near, int n_far)
{
    GensetShape g;
    const int cap = k_near + n_far;
    g.cap1 = cap > 0 ? (size_t)cap : 1;
    g.np1 = NP > 0 ? (size_t)NP : 1;
    long long n2 = 2048;
    while (n2 < NP) n2 <<= 1;
    g.n2 = (size_t)n2;
    g.strata = (size_t)std::max(1, k_near);
    int batch = 4096;
    while (batch < 4 * cap && batch < 65536) batch <<= 1;
    g.batch = batch;
    g.scan_tmp_len = scan_tmp_needed((int)std::max<long long>(NP, 1));
    return g;
}

size_t round256(size_t b) { return ((b ? b : 16) + 255) & ~(size_t)255; }

}  // namespace

uint64_t genset_bytes(long long NP, int k_near, int n_far)
{
    GensetShape g = genset_shape(NP, k_near, n_far);
    size_t c = g.cap1, n = g.np1, b = (size_t)g.batch;
    size_t sizes[] = {c * 4, c * 4, c * 4, c * 4, c * 4, c * 4, c * 4, c * 4, c * 4, c * 4, 4, 3 * c * 16,
                      n, g.n2 * 8, n * 4, n * 4, g.strata * 4, c * 4, c * 4, sizeof(GenState), n * 8, (n + 1) * 8,
                      3 * c * 8, 3 * c * 8, b * 4, 9 * b * 8, 9 * b * 8, 3 * b * 4, 3 * b * 4,
                      (size_t)g.scan_tmp_len * 8};
    uint64_t total = 0;
    for (size_t x : sizes) total += round256(x);
    return total;
}

int alloc_genset(vplg_context* ctx, SceneObj* so, uint64_t scene_id, PatchIndex* pi, const vplg_gen_params* p,
                 VplSetObj** out)
{
    const long long NP = pi->total;
    GensetShape g = genset_shape(NP, p->k_near, p->n_far);
    auto* v = new VplSetObj;
    v->generated = true;
    v->k_near = p->k_near;
    v->n_far = p->n_far;
    v->n_tris = so->dev.n_tris;
    v->scene_id = scene_id;
    v->patch_h = p->patch_h;
    DevVpls& dv = v->dev;
    GenBuffers& b = v->gen;
    std::memset(&b, 0, sizeof b);
    b.n_patches = (int)NP;
    b.level = pi->level;
    b.patch_off = pi->off;
    b.batch = g.batch;
    b.scan_tmp_len = g.scan_tmp_len;
    const size_t c = g.cap1, n = g.np1, bt = (size_t)g.batch;
    int rc;
    auto A = [&](auto** ptr, size_t k) { return dalloc_n(ctx, v->allocs, v->bytes, k, ptr); };
    if ((rc = A(&dv.px, c)) || (rc = A(&dv.py, c)) || (rc = A(&dv.pz, c)) || (rc = A(&dv.nx, c)) ||
        (rc = A(&dv.ny, c)) || (rc = A(&dv.nz, c)) || (rc = A(&dv.ir, c)) || (rc = A(&dv.ig, c)) ||
        (rc = A(&dv.ib, c)) || (rc = A(&dv.tri, c)) || (rc = A(&dv.count, 1)) || (rc = A(&dv.pack, 3 * c)) ||
        (rc = A(&b.pflags, n)) || (rc = A(&b.sortbuf, g.n2)) || (rc = A(&b.sorted, n)) || (rc = A(&b.keys, n)) ||
        (rc = A(&b.strata, g.strata)) || (rc = A(&b.vpl_path, c)) || (rc = A(&b.vpl_bounce, c)) ||
        (rc = A(&b.state, 1)) || (rc = A(&b.q, n)) || (rc = A(&b.scan_out, n + 1)) ||
        (rc = A(&b.stage_pos, 3 * c)) || (rc = A(&b.stage_flux, 3 * c)) || (rc = A(&b.w_count, bt)) ||
        (rc = A(&b.w_pos, 9 * bt)) || (rc = A(&b.w_flux, 9 * bt)) || (rc = A(&b.w_tri, 3 * bt)) ||
        (rc = A(&b.w_bounce, 3 * bt)) || (rc = A(&b.scan_tmp, (size_t)b.scan_tmp_len))) {
        release_set(ctx, v);
        return rc;
    }
    dv.capacity = p->k_near + p->n_far;
    b.F = b.scan_out + 1;
    hipError_t e = hipEventCreateWithFlags(&v->done, hipEventDisableTiming);
    if (e != hipSuccess) {
        v->done = nullptr;
        release_set(ctx, v);
        return fail(VPLG_EHIP, "event: %s", hipGetErrorString(e));
    }
    *out = v;
    return VPLG_OK;
}

int launch_genset(SceneObj* so, VplSetObj* v, const vplg_camera* cam, const vplg_gen_params* p, hipStream_t s)
{
    CamBasis cb = cam_basis(cam);
    GenParams gp{p->k_near,  p->n_far,     p->max_bounces, p->max_paths,  p->d_near,       p->patch_h,
                 p->t_eps,   p->walk_near, p->jitter,      p->brightness, p->walk_schedule};
    HIPCHK(launch_generate(so->dev, so->light, cb, gp, v->dev, v->gen, s));
    const bool radii = so->dev.n_tris >= kFreeMinTris;
    HIPCHK(launch_pack_vpls(radii ? &so->dev : nullptr, v->dev, s));
    v->radius_scene = radii ? so->id : 0;
    HIPCHK(hipEventRecord(v->done, s));
    return VPLG_OK;
}

}  // namespace rt
}  // namespace vplg

extern "C" {

int vplg_gbuffer_render(vplg_context* ctx, uint64_t scene_id, const vplg_camera* cam, const vplg_gbuffer* gb,
                        void* stream)
{
    int rc = set_device(ctx);
    if (rc) return rc;
    SceneObj* so = find_scene(ctx, scene_id);
    if (!so) return fail(VPLG_ENOTFOUND, "unknown scene %llu", (unsigned long long)scene_id);
    if ((rc = check_camera(cam)) || (rc = check_gbuffer(gb))) return rc;
    if (gb->width != cam->width || gb->height != cam->height)
        return fail(VPLG_EINVAL, "gbuffer %dx%d does not match camera %dx%d", gb->width, gb->height, cam->width,
                    cam->height);
    return render_gbuffer(so, cam, gb, (hipStream_t)stream);
}

int vplg_vpls_generate(vplg_context* ctx, uint64_t scene_id, const vplg_camera* cam, const vplg_gen_params* p,
                       void* stream, uint64_t* vplset_id)
{
    int rc = set_device(ctx);
    if (rc) return rc;
    if (!vplset_id) return fail(VPLG_EINVAL, "null argument");
    SceneObj* so = find_scene(ctx, scene_id);
    if (!so) return fail(VPLG_ENOTFOUND, "unknown scene %llu", (unsigned long long)scene_id);
    if ((rc = check_camera(cam)) || (rc = check_gen_params(p))) return rc;
    hipStream_t s = (hipStream_t)stream;
    PatchIndex* pi = nullptr;
    if ((rc = patch_index(ctx, so, p->patch_h, s, &pi))) return rc;
    VplSetObj* v = nullptr;
    if ((rc = alloc_genset(ctx, so, scene_id, pi, p, &v))) return rc;
    if ((rc = launch_genset(so, v, cam, p, s))) {
        release_set(ctx, v);
        return rc;
    }
    std::lock_guard<std::recursive_mutex> lock(ctx->mu);
    uint64_t id = ctx->next_id++;
    ctx->sets[id] = v;
    *vplset_id = id;
    return VPLG_OK;
}

int vplg_vpls_regenerate(vplg_context* ctx, uint64_t vplset_id, const vplg_camera* cam, const vplg_gen_params* p,
                         void* stream)
{
    int rc = set_device(ctx);
    if (rc) return rc;
    VplSetObj* v = find_set(ctx, vplset_id);
    if (!v) return fail(VPLG_ENOTFOUND, "unknown VPL set %llu", (unsigned long long)vplset_id);
    if (!v->generated) return fail(VPLG_EINVAL, "VPL set %llu was uploaded, not generated", (unsigned long long)vplset_id);
    if ((rc = check_camera(cam)) || (rc = check_gen_params(p))) return rc;
    if (p->k_near != v->k_near || p->n_far != v->n_far || p->patch_h != v->patch_h)
        return fail(VPLG_EINVAL, "regeneration must keep k_near, n_far and patch_h of the set");
    SceneObj* so = find_scene(ctx, v->scene_id);
    if (!so) return fail(VPLG_ENOTFOUND, "the scene of VPL set %llu was released", (unsigned long long)vplset_id);
    return launch_genset(so, v, cam, p, (hipStream_t)stream);
}

int vplg_vplset_stats(vplg_context* ctx, uint64_t vplset_id, vplg_gen_stats* out)
{
    int rc = set_device(ctx);
    if (rc) return rc;
    if (!out) return fail(VPLG_EINVAL, "null argument");
    VplSetObj* v = find_set(ctx, vplset_id);
    if (!v) return fail(VPLG_ENOTFOUND, "unknown VPL set %llu", (unsigned long long)vplset_id);
    if (!v->generated) return fail(VPLG_EINVAL, "VPL set %llu was uploaded, not generated", (unsigned long long)vplset_id);
    if ((rc = wait_set(v))) return rc;
    GenState st;
    HIPCHK(hipMemcpy(&st, v->gen.state, sizeof st, hipMemcpyDeviceToHost));
    out->n_patches = st.n_patches;
    out->n_near = st.n_near;
    out->n_eligible = st.n_eligible;
    out->q_total = st.q_total;
    out->k_eff = st.k_eff;
    out->n_far_target = st.n_far_target;
    out->n_far = st.n_far;
    out->n_paths = st.n_paths;
    for (int i = 0; i < 3; ++i) out->far_by_bounce[i] = st.far_b[i];
    out->flags = st.flags;
    out->near_discarded = st.near_discarded;
    if (st.flags & 2) return fail(VPLG_EINVAL, "fixed-point area total too large for %d strata", v->k_near);
    return VPLG_OK;
}

int vplg_vplset_count(vplg_context* ctx, uint64_t vplset_id, int32_t* n)
{
    int rc = set_device(ctx);
    if (rc) return rc;
    if (!n) return fail(VPLG_EINVAL, "null argument");
    VplSetObj* v = find_set(ctx, vplset_id);
    if (!v) return fail(VPLG_ENOTFOUND, "unknown VPL set %llu", (unsigned long long)vplset_id);
    return set_count(v, n);
}

int vplg_vpls_upload(vplg_context* ctx, const float* pos, const float* nrm, const float* intensity,
                     const int32_t* host_tri, int32_t n, void* stream, uint64_t* vplset_id)
{
    int rc = set_device(ctx);
    if (rc) return rc;
    if (!vplset_id || n < 0 || (n > 0 && (!pos || !nrm || !intensity || !host_tri)))
        return fail(VPLG_EINVAL, "bad VPL upload arguments");
    if (n > (1 << 26)) return fail(VPLG_EINVAL, "too many VPLs (%d)", n);
    hipStream_t s = (hipStream_t)stream;
    auto* v = new VplSetObj;
    DevVpls& dv = v->dev;
    size_t c1 = n > 0 ? (size_t)n : 1;
    auto A = [&](auto** ptr, size_t k) { return dalloc_n(ctx, v->allocs, v->bytes, k, ptr); };
    if ((rc = A(&dv.px, c1)) || (rc = A(&dv.py, c1)) || (rc = A(&dv.pz, c1)) || (rc = A(&dv.nx, c1)) ||
        (rc = A(&dv.ny, c1)) || (rc = A(&dv.nz, c1)) || (rc = A(&dv.ir, c1)) || (rc = A(&dv.ig, c1)) ||
        (rc = A(&dv.ib, c1)) || (rc = A(&dv.tri, c1)) || (rc = A(&dv.count, 1)) || (rc = A(&dv.pack, 3 * c1))) {
        release_set(ctx, v);
        return rc;
    }
    dv.capacity = n;
    std::vector<float> planes(9 * c1);
    for (int i = 0; i < n; ++i)
        for (int k = 0; k < 3; ++k) {
            planes[k * c1 + i] = pos[3 * i + k];
            planes[(3 + k) * c1 + i] = nrm[3 * i + k];
            planes[(6 + k) * c1 + i] = intensity[3 * i + k];
        }
    float* dst[9] = {dv.px, dv.py, dv.pz, dv.nx, dv.ny, dv.nz, dv.ir, dv.ig, dv.ib};
    hipError_t e = hipSuccess;
    for (int k = 0; k < 9 && e == hipSuccess && n > 0; ++k)
        e = hipMemcpyAsync(dst[k], &planes[k * c1], (size_t)n * sizeof(float), hipMemcpyHostToDevice, s);
    if (e == hipSuccess && n > 0) e = hipMemcpyAsync(dv.tri, host_tri, (size_t)n * 4, hipMemcpyHostToDevice, s);
    int32_t cnt = n;
    if (e == hipSuccess) e = hipMemcpyAsync(dv.count, &cnt, 4, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = launch_pack_vpls(nullptr, dv, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) {
        release_set(ctx, v);
        return fail(VPLG_EHIP, "VPL upload failed: %s", hipGetErrorString(e));
    }
    std::lock_guard<std::recursive_mutex> lock(ctx->mu);
    uint64_t id = ctx->next_id++;
    ctx->sets[id] = v;
    *vplset_id = id;
    return VPLG_OK;
}

int vplg_vpls_download(vplg_context* ctx, uint64_t vplset_id, float* pos, float* nrm, float* intensity,
                       int32_t* host_tri, int32_t cap, int32_t* n)
{
    int rc = set_device(ctx);
    if (rc) return rc;
    if (!n) return fail(VPLG_EINVAL, "null count pointer");
    VplSetObj* v = find_set(ctx, vplset_id);
    if (!v) return fail(VPLG_ENOTFOUND, "unknown VPL set %llu", (unsigned long long)vplset_id);
    int32_t cnt = 0;
    if ((rc = set_count(v, &cnt))) return rc;
    *n = cnt;
    if (cap < cnt) return fail(VPLG_EINVAL, "capacity %d < %d VPLs", cap, cnt);
    if (cnt == 0) return VPLG_OK;
    std::vector<float> tmp(9 * (size_t)cnt);
    const DevVpls& dv = v->dev;
    const float* src[9] = {dv.px, dv.py, dv.pz, dv.nx, dv.ny, dv.nz, dv.ir, dv.ig, dv.ib};
    for (int k = 0; k < 9; ++k)
        HIPCHK(hipMemcpy(&tmp[k * (size_t)cnt], src[k], (size_t)cnt * 4, hipMemcpyDeviceToHost));
    for (int i = 0; i < cnt; ++i)
        for (int k = 0; k < 3; ++k) {
            if (pos) pos[3 * i + k] = tmp[k * (size_t)cnt + i];
            if (nrm) nrm[3 * i + k] = tmp[(3 + k) * (size_t)cnt + i];
            if (intensity) intensity[3 * i + k] = tmp[(6 + k) * (size_t)cnt + i];
        }
    if (host_tri) HIPCHK(hipMemcpy(host_tri, dv.tri, (size_t)cnt * 4, hipMemcpyDeviceToHost));
    return VPLG_OK;
}

int vplg_vplset_debug(vplg_context* ctx, uint64_t vplset_id, int32_t what, void* host_buf, int64_t cap_bytes,
                      int64_t* n_items)
{
    int rc = set_device(ctx);
    if (rc) return rc;
    if (!n_items) return fail(VPLG_EINVAL, "null argument");
    VplSetObj* v = find_set(ctx, vplset_id);
    if (!v) return fail(VPLG_ENOTFOUND, "unknown VPL set %llu", (unsigned long long)vplset_id);
    if (!v->generated) return fail(VPLG_EINVAL, "VPL set was uploaded, not generated");
    if ((rc = wait_set(v))) return rc;
    GenState st;
    HIPCHK(hipMemcpy(&st, v->gen.state, sizeof st, hipMemcpyDeviceToHost));
    int32_t cnt = 0;
    if ((rc = set_count(v, &cnt))) return rc;
    const void* src = nullptr;
    size_t elem = 0;
    int64_t n = 0;
    switch (what) {
    case 0: src = v->gen.pflags; elem = 1; n = st.n_patches; break;
    case 1: src = v->gen.sorted; elem = 4; n = st.n_eligible; break;
    case 2: src = v->gen.keys; elem = 4; n = st.n_eligible; break;
    case 3: src = v->gen.F; elem = 8; n = st.n_eligible; break;
    case 4: src = v->gen.strata; elem = 4; n = st.k_eff; break;
    case 5: src = v->gen.vpl_path; elem = 4; n = cnt; break;
    case 6: src = v->gen.vpl_bounce; elem = 4; n = cnt; break;
    case 7: src = v->gen.patch_off; elem = 8; n = v->n_tris + 1; break;
    default: return fail(VPLG_EINVAL, "unknown debug array %d", what);
    }
    *n_items = n;
    if (!host_buf || cap_bytes < (int64_t)(n * elem)) return fail(VPLG_EINVAL, "buffer too small (%lld bytes needed)",
                                                                   (long long)(n * elem));
    if (n > 0) HIPCHK(hipMemcpy(host_buf, src, (size_t)n * elem, hipMemcpyDeviceToHost));
    return VPLG_OK;
}

int vplg_vplset_release(vplg_context* ctx, uint64_t vplset_id)
{
    int rc = set_device(ctx);
    if (rc) return rc;
    VplSetObj* v = find_set(ctx, vplset_id);
    if (!v) return fail(VPLG_ENOTFOUND, "unknown VPL set %llu", (unsigned long long)vplset_id);
    HIPCHK(hipDeviceSynchronize());
    std::lock_guard<std::recursive_mutex> lock(ctx->mu);
    release_set(ctx, v);
    ctx->sets.erase(vplset_id);
    return VPLG_OK;
}

}  // extern "C"

namespace vplg {
namespace rt {

static uint32_t ceil_log2(long long x)
{
    uint32_t k = 0;
    while ((1ll << k) < x) ++k;
    return k;
}

uint32_t shape_bucket(int width, int height, int n_vpls)
{
    return (ceil_log2((long long)width * height) << 8) | ceil_log2(n_vpls > 0 ? n_vpls : 1);
}

TileShape tuned_shape(vplg_context* ctx, int width, int height, int n_vpls, bool batched)
{
    // a server thread resolves tile shapes while the caller may autotune
    std::lock_guard<std::recursive_mutex> lock(ctx->mu);
    const auto& table = batched ? ctx->tuned_batch : ctx->tuned;
    auto it = table.find(shape_bucket(width, height, n_vpls));
    if (it != table.end()) return it->second;
    TileShape t;
    t.px_tiles = 1;
    t.waves = 8;
    if (batched) return t;
    if (ctx->cus == 0 && hipDeviceGetAttribute(&ctx->cus, hipDeviceAttributeMultiprocessorCount, ctx->device) != hipSuccess)
        ctx->cus = 256;
    const long long tiles = (long long)((width + 7) / 8) * ((height + 7) / 8);
    t.waves = tiles < (long long)kWideTilesPerCu * ctx->cus ? 16 : 8;
    return t;
}

// px_tiles of a tile_px value (0 = 64), or 0 if it is not one of 0, 64, 128, 256
static int px_tiles_of(int tile_px) { return tile_px == 0 || tile_px == 64 ? 1 : tile_px == 128 ? 2 : tile_px == 256 ? 4 : 0; }

int gather_common(vplg_context* ctx, uint64_t scene_id, uint64_t vplset_id, const vplg_gbuffer* gb,
                  float* const radiance[3], const vplg_gather_params* p, GatherArgs* a, bool batched)
{
    int rc = set_device(ctx);
    if (rc) return rc;
    if (!radiance || !p) return fail(VPLG_EINVAL, "null argument");
    for (int c = 0; c < 3; ++c)
        if (!radiance[c]) return fail(VPLG_EINVAL, "null radiance plane");
    if ((rc = check_gbuffer(gb))) return rc;
    if (!(p->g_clamp > 0.f) || !(p->t_eps >= 0.f && p->t_eps < 0.5f))
        return fail(VPLG_EINVAL, "bad gather parameters (g_clamp %g, t_eps %g)", p->g_clamp, p->t_eps);
    SceneObj* so = find_scene(ctx, scene_id);
    if (!so) return fail(VPLG_ENOTFOUND, "unknown scene %llu", (unsigned long long)scene_id);
    VplSetObj* v = find_set(ctx, vplset_id);
    if (!v) return fail(VPLG_ENOTFOUND, "unknown VPL set %llu", (unsigned long long)vplset_id);
    return gather_args(ctx, so, v, gb, radiance, p, a, batched);
}

int gather_args(vplg_context* ctx, SceneObj* so, VplSetObj* v, const vplg_gbuffer* gb, float* const radiance[3],
                const vplg_gather_params* p, GatherArgs* a, bool batched)
{
    a->scene = so->dev;
    a->vpls = v->dev;
    a->gb = dev_gbuffer(gb);
    for (int c = 0; c < 3; ++c) a->out[c] = radiance[c];
    a->g_clamp = p->g_clamp;
    a->t_eps = p->t_eps;
    a->counters = nullptr;
    a->split_cap = 0;
    a->split_full = a->split_count = 0;
    a->split_part = nullptr;
    a->free_ends = so->dev.n_tris < kFreeMinTris ? 0 : 1 | (v->radius_scene == so->id ? 2 : 0);
    // tile_vpl: waves (VPL slices) per 8 x 8 tile, tile_px: pixels per work item; tile_vpl 0 leaves the shape
    // to the autotuned table (else the tile-count rule), with tile_px, if given, fixing the pixel block
    int G = px_tiles_of(p->tile_px);
    if (G == 0) return fail(VPLG_EINVAL, "tile_px must be 0, 64, 128 or 256 (got %d)", p->tile_px);
    int w = p->tile_vpl;
    if (w == 0) {
        const TileShape t = tuned_shape(ctx, gb->width, gb->height, v->dev.capacity, batched);
        w = t.waves;
        if (p->tile_px == 0) G = t.px_tiles;
        while (w > 1 && G * w > kGatherMaxWorkgroupWaves) w >>= 1;
    }
    if (w < 1 || w > 16 || (w & (w - 1)))
        return fail(VPLG_EINVAL, "tile_vpl must be 0 or a power of two in [1, 16] (got %d)", p->tile_vpl);
    if (G * w > kGatherMaxWorkgroupWaves)
        return fail(VPLG_EINVAL, "tile_px / 64 * tile_vpl must be at most %d (got %d * %d)", kGatherMaxWorkgroupWaves,
                    G, w);
    a->waves_per_tile = w;
    a->px_tiles = G;
    return VPLG_OK;
}

int gather_grid(vplg_context* ctx, int waves, bool counted, int* blocks)
{
    std::lock_guard<std::recursive_mutex> lk(ctx->mu);
    if (ctx->cus == 0) HIPCHK(hipDeviceGetAttribute(&ctx->cus, hipDeviceAttributeMultiprocessorCount, ctx->device));
    const int lw = __builtin_ctz((unsigned)waves);
    int& per_cu = ctx->gather_blocks[counted ? 1 : 0][lw];
    if (per_cu == 0) {
        HIPCHK(gather_occupancy(waves, counted, &per_cu));
        if (per_cu < 1) per_cu = 1;
    }
    *blocks = ctx->cus * per_cu;
    return VPLG_OK;
}

int run_gather(vplg_context* ctx, const GatherArgs& a, bool counted, hipStream_t s, bool split_tail)
{
    GatherWork wk;
    int blocks = 0;
    {
        std::lock_guard<std::recursive_mutex> lk(ctx->mu);
        auto it = ctx->stream_work.find((void*)s);
        if (it == ctx->stream_work.end()) {
            HIPCHK(hipMalloc(&wk.counter, sizeof(unsigned int)));
            hipError_t e = hipMalloc(&wk.part, sizeof(float) * (size_t)kGatherSplitCap * gather_split_floats_per_tile());
            if (e != hipSuccess) {
                (void)hipFree(wk.counter);
                return fail(VPLG_EHIP, "gather work memory: %s", hipGetErrorString(e));
            }
            ctx->stream_work[(void*)s] = wk;
        } else {
            wk = it->second;
        }
    }
    int rc = gather_grid(ctx, a.waves_per_tile * a.px_tiles, counted, &blocks);
    if (rc) return rc;
    GatherArgs b = a;
    b.split_cap = split_tail ? kGatherSplitCap : 0;
    b.split_part = wk.part;
    HIPCHK(launch_gather(b, counted, wk.counter, blocks, s));
    return VPLG_OK;
}

}  // namespace rt
}  // namespace vplg

extern "C" {

int vplg_gather(vplg_context* ctx, uint64_t scene_id, uint64_t vplset_id, const vplg_gbuffer* gb,
                float* const radiance[3], const vplg_gather_params* p, void* stream)
{
    GatherArgs a;
    int rc = gather_common(ctx, scene_id, vplset_id, gb, radiance, p, &a);
    if (rc) return rc;
    return run_gather(ctx, a, false, (hipStream_t)stream);
}

int vplg_gather_noalloc(vplg_context* ctx, uint64_t scene_id, uint64_t vplset_id, const vplg_gbuffer* gb,
                        float* const radiance[3], const vplg_gather_params* p, void* stream)
{
    GatherArgs a;
    int rc = gather_common(ctx, scene_id, vplset_id, gb, radiance, p, &a);
    if (rc) return rc;
    void* scr = gather_scratch_address(ctx->device);
    if (!scr) return fail(VPLG_EHIP, "device %d: the gather's scratch array has no address", ctx->device);
    int blocks = 0;
    if ((rc = gather_grid(ctx, a.waves_per_tile * a.px_tiles, false, &blocks))) return rc;
    // the launch splits at most gather_scratch_split_cap() tiles, whatever
    // the view's size; check the bound the array was sized for all the same
    const size_t need = 256 + sizeof(float) * (size_t)gather_scratch_split_cap() * gather_split_floats_per_tile();
    if (need > gather_scratch_bytes())
        return fail(VPLG_EINVAL, "gather scratch: %zu bytes needed, %zu available", need, gather_scratch_bytes());
    HIPCHK(launch_gather_scratch(a, scr, blocks, (hipStream_t)stream));
    return VPLG_OK;
}

int vplg_gather_counted(vplg_context* ctx, uint64_t scene_id, uint64_t vplset_id, const vplg_gbuffer* gb,
                        float* const radiance[3], const vplg_gather_params* p, uint64_t* counters, void* stream)
{
    GatherArgs a;
    int rc = gather_common(ctx, scene_id, vplset_id, gb, radiance, p, &a);
    if (rc) return rc;
    if (!counters) return fail(VPLG_EINVAL, "null counters");
    a.counters = (unsigned long long*)counters;
    return run_gather(ctx, a, true, (hipStream_t)stream);
}

int vplg_direct(vplg_context* ctx, uint64_t scene_id, const vplg_gbuffer* gb, float* const radiance[3], float t_eps,
                void* stream)
{
    int rc = set_device(ctx);
    if (rc) return rc;
    if (!radiance) return fail(VPLG_EINVAL, "null radiance");
    for (int c = 0; c < 3; ++c)
        if (!radiance[c]) return fail(VPLG_EINVAL, "null radiance plane");
    if ((rc = check_gbuffer(gb))) return rc;
    if (!(t_eps >= 0.f && t_eps < 0.5f)) return fail(VPLG_EINVAL, "bad t_eps %g", t_eps);
    SceneObj* so = find_scene(ctx, scene_id);
    if (!so) return fail(VPLG_ENOTFOUND, "unknown scene %llu", (unsigned long long)scene_id);
    DirectArgs a;
    a.scene = so->dev;
    a.light = so->light;
    a.gb = dev_gbuffer(gb);
    for (int c = 0; c < 3; ++c) a.out[c] = radiance[c];
    a.t_eps = t_eps;
    HIPCHK(launch_direct(a, (hipStream_t)stream));
    return VPLG_OK;
}

int vplg_gather_visibility_dump(vplg_context* ctx, uint64_t scene_id, uint64_t vplset_id, const vplg_gbuffer* gb,
                                const int32_t* pixels, int32_t n_px, uint32_t* vis_bits, const vplg_gather_params* p,
                                void* stream)
{
    int rc = set_device(ctx);
    if (rc) return rc;
    if ((rc = check_gbuffer(gb))) return rc;
    if (n_px < 0 || (n_px > 0 && (!pixels || !vis_bits)) || !p) return fail(VPLG_EINVAL, "bad dump arguments");
    SceneObj* so = find_scene(ctx, scene_id);
    if (!so) return fail(VPLG_ENOTFOUND, "unknown scene %llu", (unsigned long long)scene_id);
    VplSetObj* v = find_set(ctx, vplset_id);
    if (!v) return fail(VPLG_ENOTFOUND, "unknown VPL set %llu", (unsigned long long)vplset_id);
    int32_t M = 0;
    if ((rc = set_count(v, &M))) return rc;
    VisDumpArgs a;
    a.scene = so->dev;
    a.vpls = v->dev;
    a.gb = dev_gbuffer(gb);
    a.pixels = pixels;
    a.n_px = n_px;
    a.words = (M + 31) / 32;
    a.bits = vis_bits;
    a.t_eps = p->t_eps;
    a.free_ends = so->dev.n_tris < kFreeMinTris ? 0 : 1 | (v->radius_scene == so->id ? 2 : 0);
    HIPCHK(launch_vis_dump(a, (hipStream_t)stream));
    return VPLG_OK;
}

}  // extern "C"

static int batch_init(vplg_context* ctx, int wide)
{
    BatchEngine& be = ctx->batch;
    if (!be.ready) {
        HIPCHK(hipMalloc(&be.d_tab, sizeof(BatchTable)));
        HIPCHK(hipMalloc(&be.d_views, sizeof(GatherArgs) * kBatchMaxViews));
        HIPCHK(hipMalloc(&be.d_counter, sizeof(unsigned int)));
        HIPCHK(hipHostMalloc(&be.h_tab, sizeof(BatchTable), hipHostMallocDefault));
        HIPCHK(hipHostMalloc(&be.h_views, sizeof(GatherArgs) * kBatchMaxViews, hipHostMallocDefault));
        HIPCHK(hipEventCreateWithFlags(&be.staged, hipEventDisableTiming));
        HIPCHK(hipEventCreateWithFlags(&be.replayed, hipEventDisableTiming));
        HIPCHK(hipStreamCreateWithFlags(&be.capture, hipStreamNonBlocking));
        be.ready = true;
    }
    if (be.exec[wide]) return VPLG_OK;
    const int bw = wide ? kBatchWideWaves : kBatchBlockWaves;
    int cus = 0, per_cu = 0;
    HIPCHK(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, ctx->device));
    HIPCHK(gather_batch_occupancy(bw, &per_cu));
    be.blocks[wide] = cus * (per_cu > 0 ? per_cu : 1);
    // the graph holds only fixed device pointers: the table's contents change between replays
    HIPCHK(hipStreamBeginCapture(be.capture, hipStreamCaptureModeThreadLocal));
    hipError_t e = launch_gather_batch(be.d_tab, be.d_views, be.d_counter, be.blocks[wide], bw, be.capture);
    hipError_t e2 = hipStreamEndCapture(be.capture, &be.graph[wide]);
    if (e != hipSuccess) return fail(VPLG_EHIP, "batch capture: %s", hipGetErrorString(e));
    if (e2 != hipSuccess) return fail(VPLG_EHIP, "batch capture end: %s", hipGetErrorString(e2));
    HIPCHK(hipGraphInstantiate(&be.exec[wide], be.graph[wide], nullptr, nullptr, 0));
    return VPLG_OK;
}

extern "C" {

int vplg_gather_batch(vplg_context* ctx, const vplg_view* views, int32_t n_views, void* stream)
{
    int rc = set_device(ctx);
    if (rc) return rc;
    if (n_views < 0 || n_views > kBatchMaxViews || (n_views > 0 && !views))
        return fail(VPLG_EINVAL, "n_views must be in [0, %d]", kBatchMaxViews);
    if (n_views == 0) return VPLG_OK;
    // resolve and check every view before touching the staging buffers
    std::vector<GatherArgs> args(n_views);
    std::vector<int> waves(n_views), items(n_views);
    std::vector<double> cost(n_views);
    int wide = 0;
    for (int v = 0; v < n_views; ++v) {
        const vplg_view& vw = views[v];
        if ((rc = gather_common(ctx, vw.scene_id, vw.vplset_id, &vw.gb, vw.radiance, &vw.params, &args[v], true)))
            return fail(rc, "view %d: %s", v, g_err.c_str());
        waves[v] = args[v].waves_per_tile;
        if (waves[v] * args[v].px_tiles > kBatchBlockWaves) wide = 1;
        cost[v] = (double)vw.gb.width * vw.gb.height * (double)args[v].vpls.capacity;
    }
    // one workgroup size per launch: 16 waves when some view's pixel block
    // needs more than 8 (its tiles times its waves per tile)
    const int bw = wide ? kBatchWideWaves : kBatchBlockWaves;
    for (int v = 0; v < n_views; ++v) {
        const int blocks = gather_view_blocks(views[v].gb.width, views[v].gb.height, args[v].px_tiles);
        const int per_item = bw / waves[v] / args[v].px_tiles;  // blocks per workgroup item
        items[v] = (blocks + per_item - 1) / per_item;
    }
    if ((rc = batch_init(ctx, wide))) return rc;
    BatchEngine& be = ctx->batch;
    // most expensive views first (their tiles are claimed first), ties by index
    std::vector<int> order(n_views);
    for (int v = 0; v < n_views; ++v) order[v] = v;
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return cost[a] > cost[b]; });
    HIPCHK(hipEventSynchronize(be.staged));  // the previous call's copies have read the staging
    long long total = 0;
    for (int i = 0; i < n_views; ++i) {
        int v = order[i];
        be.h_tab->prefix[i] = (int)total;
        be.h_tab->waves[i] = waves[v];
        be.h_views[i] = args[v];
        total += items[v];
    }
    if (total > 0x7fffffff) return fail(VPLG_EINVAL, "batch too large");
    be.h_tab->prefix[n_views] = (int)total;
    be.h_tab->n_views = n_views;
    hipStream_t s = (hipStream_t)stream;
    // the device table, views and counter are shared by every call: this
    // call's copies wait for the previous replay, whatever stream it ran on
    HIPCHK(hipStreamWaitEvent(s, be.replayed, 0));
    HIPCHK(hipMemcpyAsync(be.d_tab, be.h_tab, sizeof(BatchTable), hipMemcpyHostToDevice, s));
    HIPCHK(hipMemcpyAsync(be.d_views, be.h_views, sizeof(GatherArgs) * n_views, hipMemcpyHostToDevice, s));
    HIPCHK(hipEventRecord(be.staged, s));
    HIPCHK(hipGraphLaunch(be.exec[wide], s));
    HIPCHK(hipEventRecord(be.replayed, s));
    return VPLG_OK;
}

int vplg_autotune(vplg_context* ctx, uint64_t scene_id, uint64_t vplset_id, const vplg_gbuffer* gb,
                  float* const radiance[3], const vplg_gather_params* p, void* stream, int32_t* best_tile_vpl,
                  int32_t* best_tile_px)
{
    if (!p || !best_tile_vpl || !best_tile_px) return fail(VPLG_EINVAL, "null argument");
    hipStream_t s = (hipStream_t)stream;
    hipEvent_t e0, e1;
    HIPCHK(hipEventCreate(&e0));
    HIPCHK(hipEventCreate(&e1));
    float best_ms = 1e30f;
    TileShape best;
    int n_vpls = 0;
    for (int G = 1; G <= 4; G <<= 1) {
        for (int w = 1; G * w <= kGatherMaxWorkgroupWaves; w <<= 1) {
            vplg_gather_params q = *p;
            q.tile_vpl = w;
            q.tile_px = 64 * G;
            GatherArgs a;
            int rc = gather_common(ctx, scene_id, vplset_id, gb, radiance, &q, &a);
            if (rc) {
                (void)hipEventDestroy(e0);
                (void)hipEventDestroy(e1);
                return rc;
            }
            n_vpls = a.vpls.capacity;
            float ms = 0.f;
            rc = run_gather(ctx, a, false, s);  // warm
            hipError_t e = hipSuccess;
            if (!rc) e = hipEventRecord(e0, s);
            if (!rc && e == hipSuccess) rc = run_gather(ctx, a, false, s);
            if (!rc && e == hipSuccess) e = hipEventRecord(e1, s);
            if (!rc && e == hipSuccess) e = hipEventSynchronize(e1);
            if (!rc && e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
            if (rc || e != hipSuccess) {
                (void)hipEventDestroy(e0);
                (void)hipEventDestroy(e1);
                return rc ? rc : fail(VPLG_EHIP, "autotune: %s", hipGetErrorString(e));
            }
            if (ms < best_ms) {
                best_ms = ms;
                best.waves = w;
                best.px_tiles = G;
            }
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    {
        std::lock_guard<std::recursive_mutex> lock(ctx->mu);
        ctx->tuned[shape_bucket(gb->width, gb->height, n_vpls)] = best;
    }
    *best_tile_vpl = best.waves;
    *best_tile_px = 64 * best.px_tiles;
    return VPLG_OK;
}

// Time one batched launch of `views` on `s` (the caller has synchronised s).
static int time_batch(vplg_context* ctx, const std::vector<vplg_view>& views, hipStream_t s, hipEvent_t e0,
                      hipEvent_t e1, float* ms)
{
    HIPCHK(hipEventRecord(e0, s));
    int rc = vplg_gather_batch(ctx, views.data(), (int32_t)views.size(), s);
    if (rc) return rc;
    HIPCHK(hipEventRecord(e1, s));
    HIPCHK(hipEventSynchronize(e1));
    HIPCHK(hipEventElapsedTime(ms, e0, e1));
    return VPLG_OK;
}

int vplg_autotune_batch(vplg_context* ctx, const vplg_view* views, int32_t n_views, void* stream, int32_t* n_tuned)
{
    int rc = set_device(ctx);
    if (rc) return rc;
    if (n_views < 0 || n_views > kBatchMaxViews || (n_views > 0 && !views) || !n_tuned)
        return fail(VPLG_EINVAL, "bad autotune_batch arguments");
    *n_tuned = 0;
    hipStream_t s = (hipStream_t)stream;
    // the open views (tile_vpl 0, tile_px 0), by shape bucket; the rest stay as given
    std::map<uint32_t, std::vector<int>> bucket;
    std::map<uint32_t, double> bucket_cost;
    for (int v = 0; v < n_views; ++v) {
        GatherArgs a;
        if ((rc = gather_common(ctx, views[v].scene_id, views[v].vplset_id, &views[v].gb, views[v].radiance,
                                &views[v].params, &a, true)))
            return fail(rc, "view %d: %s", v, g_err.c_str());
        if (views[v].params.tile_vpl != 0 || views[v].params.tile_px != 0) continue;
        const uint32_t k = shape_bucket(views[v].gb.width, views[v].gb.height, a.vpls.capacity);
        bucket[k].push_back(v);
        bucket_cost[k] += (double)views[v].gb.width * views[v].gb.height * (double)a.vpls.capacity;
    }
    std::vector<uint32_t> keys;
    for (auto& kv : bucket) keys.push_back(kv.first);
    std::stable_sort(keys.begin(), keys.end(), [&](uint32_t a, uint32_t b) { return bucket_cost[a] > bucket_cost[b]; });
    hipEvent_t e0, e1;
    HIPCHK(hipEventCreate(&e0));
    HIPCHK(hipEventCreate(&e1));
    auto done = [&](int code) {
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        return code;
    };
    HIPCHK(hipStreamSynchronize(s));
    std::map<uint32_t, TileShape> chosen;
    for (uint32_t k : keys) {
        // the bucket's views as a batch of their own, in each shape; the first
        // run (untimed) warms the workgroup variants and the caches
        float best_ms = 1e30f;
        TileShape best;
        bool warm = false;
        for (int G = 1; G <= 4; G <<= 1) {
            for (int w = 1; G * w <= kBatchWideWaves; w <<= 1) {
                std::vector<vplg_view> sub;
                for (int v : bucket[k]) {
                    vplg_view x = views[v];
                    x.params.tile_vpl = w;
                    x.params.tile_px = 64 * G;
                    sub.push_back(x);
                }
                float ms = 0.f;
                if (!warm) {
                    if ((rc = time_batch(ctx, sub, s, e0, e1, &ms))) return done(rc);
                    warm = true;
                }
                if ((rc = time_batch(ctx, sub, s, e0, e1, &ms))) return done(rc);
                if (ms < best_ms) {
                    best_ms = ms;
                    best.waves = w;
                    best.px_tiles = G;
                }
            }
        }
        chosen[k] = best;
    }
    // keep the tuned shapes only if the whole batch runs faster with them than untuned
    std::map<uint32_t, TileShape> before;
    {
        std::lock_guard<std::recursive_mutex> lock(ctx->mu);
        before = ctx->tuned_batch;
        for (uint32_t k : keys) ctx->tuned_batch.erase(k);
    }
    std::vector<vplg_view> all(views, views + n_views);
    float ms_untuned = 0.f, ms_tuned = 0.f;
    if ((rc = time_batch(ctx, all, s, e0, e1, &ms_untuned))) return done(rc);
    if ((rc = time_batch(ctx, all, s, e0, e1, &ms_untuned))) return done(rc);
    {
        std::lock_guard<std::recursive_mutex> lock(ctx->mu);
        for (auto& kv : chosen) ctx->tuned_batch[kv.first] = kv.second;
    }
    if ((rc = time_batch(ctx, all, s, e0, e1, &ms_tuned))) return done(rc);
    if ((rc = time_batch(ctx, all, s, e0, e1, &ms_tuned))) return done(rc);
    if (ms_tuned > ms_untuned) {
        std::lock_guard<std::recursive_mutex> lock(ctx->mu);
        ctx->tuned_batch = before;
        for (uint32_t k : keys) ctx->tuned_batch.erase(k);
    } else {
        *n_tuned = (int32_t)chosen.size();
    }
    return done(VPLG_OK);
}

int vplg_autotune_lookup(vplg_context* ctx, int32_t width, int32_t height, int32_t n_vpls, int32_t batched,
                         int32_t* tile_vpl, int32_t* tile_px)
{
    if (!ctx || !tile_vpl || !tile_px) return fail(VPLG_EINVAL, "null argument");
    const TileShape t = tuned_shape(ctx, width, height, n_vpls, batched != 0);
    *tile_vpl = t.waves;
    *tile_px = 64 * t.px_tiles;
    return VPLG_OK;
}

int vplg_autotune_save(vplg_context* ctx, const char* path)
{
    if (!ctx || !path) return fail(VPLG_EINVAL, "null argument");
    FILE* f = std::fopen(path, "w");
    if (!f) return fail(VPLG_EINVAL, "cannot write %s", path);
    std::fprintf(f, "vplg-autotune 2\n");
    {
        std::lock_guard<std::recursive_mutex> lock(ctx->mu);
        for (int b = 0; b < 2; ++b)
            for (auto& kv : b ? ctx->tuned_batch : ctx->tuned)
                std::fprintf(f, "%d %u %u %d %d\n", b, kv.first >> 8, kv.first & 0xff, kv.second.waves,
                             64 * kv.second.px_tiles);
    }
    std::fclose(f);
    return VPLG_OK;
}

int vplg_autotune_load(vplg_context* ctx, const char* path)
{
    if (!ctx || !path) return fail(VPLG_EINVAL, "null argument");
    FILE* f = std::fopen(path, "r");
    if (!f) return fail(VPLG_ENOTFOUND, "cannot read %s", path);
    int version = 0;
    if (std::fscanf(f, "vplg-autotune %d", &version) != 1 || version != 2) {
        std::fclose(f);
        return fail(VPLG_EINVAL, "%s is not an autotune cache (version 2)", path);
    }
    int b, w, px;
    unsigned lp, nv;
    std::map<uint32_t, TileShape> t[2];
    while (std::fscanf(f, "%d %u %u %d %d", &b, &lp, &nv, &w, &px) == 5) {
        const int G = px_tiles_of(px);
        if ((b != 0 && b != 1) || lp > 63 || nv > 255 || w < 1 || w > 16 || (w & (w - 1)) || px == 0 || G == 0 ||
            G * w > (b ? kBatchWideWaves : kGatherMaxWorkgroupWaves)) {
            std::fclose(f);
            return fail(VPLG_EINVAL, "bad autotune entry in %s", path);
        }
        TileShape ts;
        ts.waves = w;
        ts.px_tiles = G;
        t[b][(lp << 8) | nv] = ts;
    }
    std::fclose(f);
    std::lock_guard<std::recursive_mutex> lock(ctx->mu);
    for (auto& kv : t[0]) ctx->tuned[kv.first] = kv.second;
    for (auto& kv : t[1]) ctx->tuned_batch[kv.first] = kv.second;
    return VPLG_OK;
}

}  // extern "C"
