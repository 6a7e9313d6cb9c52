// Render server: continuous admission of gather requests under an HBM budget.
//
// A server thread owns N HIP streams (default priority).  Requests queue in
// arrival order; the thread admits the queue head as soon as a slot
// (max_inflight) and enough budgeted device memory are free, and enqueues the
// request's whole chain -- G-buffer, VPL generation, gather -- on one of its
// streams, so requests that arrive while others run join them on the device.
// Completion is observed through one event per request.  Per-request device
// memory (a G-buffer block and a generated VPL set) is pooled: a finished
// request's buffers are reused by the next request of the same shape without
// any allocation or free (hipFree would synchronise the device); idle pool
// entries are freed only to make room for a request of another shape.
// A request's radiance depends only on the request (same kernels, same tile
// shape), never on what else is in flight.
#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <thread>
#include <vector>

#include "runtime_internal.h"
#include "server_pool.h"

using namespace vplg;
using namespace vplg::rt;

namespace {

int64_t now_ns()
{
    return std::chrono::duration_cast<std::chrono::nanoseconds>(std::chrono::steady_clock::now().time_since_epoch())
        .count();
}

struct ReqObj {
    uint64_t ticket = 0;
    vplg_request r;
    int state = VPLG_REQ_QUEUED;
    int error = 0;
    int64_t t_submit = 0, t_admit = 0, t_done = 0;
    uint64_t gb_bytes = 0, set_bytes = 0;
    int set_idx = -1, gb_idx = -1;
    int stream_idx = 0;
    hipEvent_t done = nullptr;
};

}  // namespace

struct vplg_server {
    vplg_context* ctx = nullptr;
    vplg_server_params prm;
    std::thread th;
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<ReqObj*> queue;
    std::vector<ReqObj*> running;
    std::map<uint64_t, ReqObj*> reqs;
    std::vector<pool::Set> sets;  // Set::v is a VplSetObj*
    std::vector<pool::Gb> gbufs;
    std::vector<hipStream_t> streams;
    int next_stream = 0;
    uint64_t next_ticket = 1;
    uint64_t used = 0;  // pooled bytes, busy or idle
    bool stopping = false;
    vplg_server_stats st;
};

namespace {

// Reserve pooled buffers for the queue head; false if they do not fit yet.
// The entries the request reuses are held before anything is freed: eviction
// only ever frees other idle entries.
bool reserve(vplg_server* s, ReqObj* q)
{
    const pool::Want w{q->r.scene_id, q->r.gen.k_near, q->r.gen.n_far, q->r.gen.patch_h, q->gb_bytes, q->set_bytes};
    const pool::Plan p = pool::plan(s->sets, s->gbufs, s->used, s->prm.hbm_budget_bytes, w);
    if (!p.fits) return false;
    for (int i : p.evict_sets) {
        release_set(s->ctx, (VplSetObj*)s->sets[i].v);
        s->used -= s->sets[i].bytes;
        s->sets[i].v = nullptr;
    }
    for (int i : p.evict_gbs) {
        (void)hipFree(s->gbufs[i].mem);
        s->used -= s->gbufs[i].bytes;
        s->gbufs[i].mem = nullptr;
    }
    int si = p.set, gi = p.gb;
    if (si < 0) {
        SceneObj* so = find_scene(s->ctx, q->r.scene_id);
        PatchIndex* pi = nullptr;
        VplSetObj* v = nullptr;
        if (!so || patch_index(s->ctx, so, q->r.gen.patch_h, s->streams[0], &pi) ||
            alloc_genset(s->ctx, so, q->r.scene_id, pi, &q->r.gen, &v)) {
            q->error = so ? VPLG_ENOMEM : VPLG_ENOTFOUND;
            return true;  // admitted as failed
        }
        pool::Set e;
        e.v = v;
        e.bytes = v->bytes;
        e.scene = q->r.scene_id;
        e.k = q->r.gen.k_near;
        e.n = q->r.gen.n_far;
        e.h = q->r.gen.patch_h;
        s->used += e.bytes;
        for (int i = 0; i < (int)s->sets.size(); ++i)
            if (!s->sets[i].v) si = i;
        if (si < 0) {
            s->sets.push_back(e);
            si = (int)s->sets.size() - 1;
        } else {
            s->sets[si] = e;
        }
    }
    if (gi < 0) {
        pool::Gb g;
        g.bytes = q->gb_bytes;
        if (hipMalloc(&g.mem, g.bytes) != hipSuccess) {
            (void)hipGetLastError();
            q->error = VPLG_ENOMEM;
            return true;  // admitted as failed (a new set stays in the pool, idle)
        }
        s->used += g.bytes;
        for (int i = 0; i < (int)s->gbufs.size(); ++i)
            if (!s->gbufs[i].mem) gi = i;
        if (gi < 0) {
            s->gbufs.push_back(g);
            gi = (int)s->gbufs.size() - 1;
        } else {
            s->gbufs[gi] = g;
        }
    }
    s->sets[si].busy = true;
    s->gbufs[gi].busy = true;
    q->set_idx = si;
    q->gb_idx = gi;
    s->st.peak_bytes = std::max<uint64_t>(s->st.peak_bytes, s->used);
    return true;
}

void release_slots(vplg_server* s, ReqObj* q)
{
    if (q->set_idx >= 0) s->sets[q->set_idx].busy = false;
    if (q->gb_idx >= 0) s->gbufs[q->gb_idx].busy = false;
    q->set_idx = q->gb_idx = -1;
}

// Enqueue the request's chain on one of the server's streams.
int launch(vplg_server* s, ReqObj* q)
{
    const vplg_request& r = q->r;
    const int W = r.camera.width, H = r.camera.height;
    const size_t P = (size_t)W * H;
    char* base = (char*)s->gbufs[q->gb_idx].mem;
    VplSetObj* v = (VplSetObj*)s->sets[q->set_idx].v;
    if (!base || !v) return fail(VPLG_EHIP, "server pool entry without memory");  // never launch on it
    vplg_gbuffer gb;
    for (int c = 0; c < 3; ++c) {
        gb.pos[c] = (float*)(base + (0 + c) * P * 4);
        gb.nrm[c] = (float*)(base + (3 + c) * P * 4);
        gb.alb[c] = (float*)(base + (6 + c) * P * 4);
    }
    gb.tri = (int32_t*)(base + 9 * P * 4);
    gb.width = W;
    gb.height = H;
    q->stream_idx = s->next_stream;
    s->next_stream = (s->next_stream + 1) % (int)s->streams.size();
    hipStream_t st = s->streams[q->stream_idx];
    SceneObj* so = find_scene(s->ctx, r.scene_id);
    if (!so) return VPLG_ENOTFOUND;
    int rc;
    if ((rc = render_gbuffer(so, &r.camera, &gb, st))) return rc;
    if ((rc = launch_genset(so, v, &r.camera, &r.gen, st))) return rc;
    GatherArgs a;
    if ((rc = gather_args(s->ctx, so, v, &gb, r.radiance, &r.gather, &a))) return rc;
    // requests overlap on the device, so no one view's tail idles it: whole
    // tiles only (split tails slowed the served p99 by about 20 ms)
    if ((rc = run_gather(s->ctx, a, false, st, false))) return rc;
    if (hipEventRecord(q->done, st) != hipSuccess) return VPLG_EHIP;
    return VPLG_OK;
}

void finish(vplg_server* s, ReqObj* q, int state, int error)
{
    q->state = state;
    q->error = error;
    q->t_done = now_ns();
    release_slots(s, q);
    if (state == VPLG_REQ_DONE) s->st.completed++;
    else if (state == VPLG_REQ_FAILED) s->st.failed++;
    else if (state == VPLG_REQ_CANCELLED) s->st.cancelled++;
}

void server_loop(vplg_server* s)
{
    (void)hipSetDevice(s->ctx->device);
    std::unique_lock<std::mutex> lock(s->mu);
    while (true) {
        bool changed = false;
        // completions
        for (size_t i = 0; i < s->running.size();) {
            ReqObj* q = s->running[i];
            hipError_t e = hipEventQuery(q->done);
            if (e == hipErrorNotReady) {
                ++i;
                continue;
            }
            finish(s, q, e == hipSuccess ? VPLG_REQ_DONE : VPLG_REQ_FAILED, e == hipSuccess ? 0 : VPLG_EHIP);
            s->running.erase(s->running.begin() + i);
            changed = true;
        }
        // admission, in arrival order
        while (!s->queue.empty() && (int)s->running.size() < s->prm.max_inflight) {
            ReqObj* q = s->queue.front();
            if (!reserve(s, q)) break;
            s->queue.pop_front();
            q->t_admit = now_ns();
            s->st.admitted++;
            int rc = q->error ? q->error : launch(s, q);
            if (rc) {
                // part of the chain may be queued: let it drain before the buffers return to the pool
                if (!q->error) (void)hipStreamSynchronize(s->streams[q->stream_idx]);
                finish(s, q, VPLG_REQ_FAILED, rc);
            } else {
                q->state = VPLG_REQ_RUNNING;
                s->running.push_back(q);
                s->st.peak_running = std::max<int64_t>(s->st.peak_running, (int64_t)s->running.size());
            }
            changed = true;
        }
        if (changed) s->cv_done.notify_all();
        if (s->stopping && s->queue.empty() && s->running.empty()) break;
        if (s->running.empty())
            s->cv_work.wait_for(lock, std::chrono::milliseconds(5));
        else
            s->cv_work.wait_for(lock, std::chrono::microseconds(50));
    }
    s->cv_done.notify_all();
}

ReqObj* find_req(vplg_server* s, uint64_t t)
{
    auto it = s->reqs.find(t);
    return it == s->reqs.end() ? nullptr : it->second;
}

void fill_timing(const ReqObj* q, vplg_timing* t)
{
    if (!t) return;
    t->state = q->state;
    t->error = q->error;
    t->submit_ns = q->t_submit;
    t->admit_ns = q->t_admit;
    t->done_ns = q->t_done;
}

}  // namespace

extern "C" {

int vplg_server_start(vplg_context* ctx, const vplg_server_params* p, vplg_server** out)
{
    int rc = set_device(ctx);
    if (rc) return rc;
    if (!p || !out) return fail(VPLG_EINVAL, "null argument");
    if (p->hbm_budget_bytes == 0 || p->max_inflight < 1 || p->max_inflight > 256 || p->n_streams < 1 ||
        p->n_streams > 16)
        return fail(VPLG_EINVAL, "bad server parameters (budget > 0, 1 <= max_inflight <= 256, 1 <= streams <= 16)");
    auto* s = new vplg_server;
    s->ctx = ctx;
    s->prm = *p;
    std::memset(&s->st, 0, sizeof s->st);
    for (int i = 0; i < p->n_streams; ++i) {
        hipStream_t st;
        if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) {
            for (auto x : s->streams) (void)hipStreamDestroy(x);
            delete s;
            return fail(VPLG_EHIP, "stream creation failed");
        }
        s->streams.push_back(st);
    }
    s->th = std::thread(server_loop, s);
    *out = s;
    return VPLG_OK;
}

int vplg_server_submit(vplg_server* s, const vplg_request* r, uint64_t* ticket)
{
    if (!s || !r || !ticket) return fail(VPLG_EINVAL, "null argument");
    int rc;
    if ((rc = set_device(s->ctx))) return rc;
    if ((rc = check_camera(&r->camera)) || (rc = check_gen_params(&r->gen))) return rc;
    for (int c = 0; c < 3; ++c)
        if (!r->radiance[c]) return fail(VPLG_EINVAL, "null radiance plane");
    if (!(r->gather.g_clamp > 0.f) || !(r->gather.t_eps >= 0.f && r->gather.t_eps < 0.5f))
        return fail(VPLG_EINVAL, "bad gather parameters");
    if (r->gather.tile_vpl < 0 || r->gather.tile_vpl > 16 || (r->gather.tile_vpl & (r->gather.tile_vpl - 1)))
        return fail(VPLG_EINVAL, "tile_vpl must be 0 or a power of two <= 16");
    SceneObj* so = find_scene(s->ctx, r->scene_id);
    if (!so) return fail(VPLG_ENOTFOUND, "unknown scene %llu", (unsigned long long)r->scene_id);
    PatchIndex* pi = nullptr;
    if ((rc = patch_index(s->ctx, so, r->gen.patch_h, s->streams[0], &pi))) return rc;
    auto* q = new ReqObj;
    q->r = *r;
    q->gb_bytes = 40ull * (uint64_t)r->camera.width * (uint64_t)r->camera.height;
    q->set_bytes = genset_bytes(pi->total, r->gen.k_near, r->gen.n_far);
    if (q->gb_bytes + q->set_bytes > s->prm.hbm_budget_bytes) {
        uint64_t need = q->gb_bytes + q->set_bytes;
        delete q;
        return fail(VPLG_EBUDGET, "request needs %llu bytes, server budget is %llu", (unsigned long long)need,
                    (unsigned long long)s->prm.hbm_budget_bytes);
    }
    if (hipEventCreateWithFlags(&q->done, hipEventDisableTiming) != hipSuccess) {
        delete q;
        return fail(VPLG_EHIP, "event creation failed");
    }
    q->t_submit = now_ns();
    {
        std::lock_guard<std::mutex> lock(s->mu);
        if (s->stopping) {
            (void)hipEventDestroy(q->done);
            delete q;
            return fail(VPLG_ECANCELLED, "server is stopping");
        }
        q->ticket = s->next_ticket++;
        s->reqs[q->ticket] = q;
        s->queue.push_back(q);
        s->st.submitted++;
        *ticket = q->ticket;
    }
    s->cv_work.notify_all();
    return VPLG_OK;
}

int vplg_server_poll(vplg_server* s, uint64_t ticket, vplg_timing* t)
{
    if (!s) return fail(VPLG_EINVAL, "null server");
    std::lock_guard<std::mutex> lock(s->mu);
    ReqObj* q = find_req(s, ticket);
    if (!q) return fail(VPLG_ENOTFOUND, "unknown ticket %llu", (unsigned long long)ticket);
    fill_timing(q, t);
    return VPLG_OK;
}

int vplg_server_wait(vplg_server* s, uint64_t ticket, int64_t timeout_ms, vplg_timing* t)
{
    if (!s) return fail(VPLG_EINVAL, "null server");
    std::unique_lock<std::mutex> lock(s->mu);
    ReqObj* q = find_req(s, ticket);
    if (!q) return fail(VPLG_ENOTFOUND, "unknown ticket %llu", (unsigned long long)ticket);
    auto final_state = [&] { return q->state >= VPLG_REQ_DONE; };
    if (timeout_ms < 0)
        s->cv_done.wait(lock, final_state);
    else if (!s->cv_done.wait_for(lock, std::chrono::milliseconds(timeout_ms), final_state)) {
        fill_timing(q, t);
        return fail(VPLG_ETIMEOUT, "ticket %llu not finished after %lld ms", (unsigned long long)ticket,
                    (long long)timeout_ms);
    }
    fill_timing(q, t);
    return q->state == VPLG_REQ_DONE ? VPLG_OK : fail(q->error ? q->error : VPLG_ECANCELLED, "request failed");
}

int vplg_server_cancel(vplg_server* s, uint64_t ticket)
{
    if (!s) return fail(VPLG_EINVAL, "null server");
    std::lock_guard<std::mutex> lock(s->mu);
    ReqObj* q = find_req(s, ticket);
    if (!q) return fail(VPLG_ENOTFOUND, "unknown ticket %llu", (unsigned long long)ticket);
    if (q->state != VPLG_REQ_QUEUED) return fail(VPLG_EBUSY, "ticket %llu is already admitted", (unsigned long long)ticket);
    s->queue.erase(std::find(s->queue.begin(), s->queue.end(), q));
    finish(s, q, VPLG_REQ_CANCELLED, VPLG_ECANCELLED);
    s->cv_done.notify_all();
    return VPLG_OK;
}

int vplg_server_query(vplg_server* s, vplg_server_stats* out)
{
    if (!s || !out) return fail(VPLG_EINVAL, "null argument");
    std::lock_guard<std::mutex> lock(s->mu);
    *out = s->st;
    out->queued = (int64_t)s->queue.size();
    out->running = (int64_t)s->running.size();
    out->pool_bytes = s->used;
    return VPLG_OK;
}

int vplg_server_stop(vplg_server* s)
{
    if (!s) return fail(VPLG_EINVAL, "null server");
    {
        std::lock_guard<std::mutex> lock(s->mu);
        s->stopping = true;
        // queued requests are cancelled; admitted ones finish
        while (!s->queue.empty()) {
            finish(s, s->queue.front(), VPLG_REQ_CANCELLED, VPLG_ECANCELLED);
            s->queue.pop_front();
        }
    }
    s->cv_work.notify_all();
    s->th.join();
    (void)hipSetDevice(s->ctx->device);
    for (auto st : s->streams) (void)hipStreamSynchronize(st);
    for (auto& p : s->sets)
        if (p.v) release_set(s->ctx, (VplSetObj*)p.v);
    for (auto& g : s->gbufs)
        if (g.mem) (void)hipFree(g.mem);
    for (auto& kv : s->reqs) {
        if (kv.second->done) (void)hipEventDestroy(kv.second->done);
        delete kv.second;
    }
    for (auto st : s->streams) (void)hipStreamDestroy(st);
    delete s;
    return VPLG_OK;
}

}  // extern "C"
