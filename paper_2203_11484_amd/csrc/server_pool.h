// Pool bookkeeping of the render server, free of device calls (the host
// tests drive it directly): which pooled entries a request reuses and which
// idle entries are evicted so that its new buffers fit the budget.
#pragma once

#include <cstdint>
#include <vector>

namespace vplg {
namespace pool {

// A pooled VPL set (v: the library's set object, opaque here) of one
// (scene, K, N_far, patch size) shape, and a pooled G-buffer block.  An
// entry is live while v / mem is set, and busy while a request holds it.
struct Set {
    void* v = nullptr;
    uint64_t bytes = 0;
    uint64_t scene = 0;
    int k = 0, n = 0;
    double h = 0.0;
    bool busy = false;
};

struct Gb {
    void* mem = nullptr;
    uint64_t bytes = 0;
    bool busy = false;
};

// What a request asks for: a set of its shape and a G-buffer block of
// gb_bytes (a block of up to twice that size is reused).
struct Want {
    uint64_t scene;
    int k, n;
    double h;
    uint64_t gb_bytes, set_bytes;
};

// Admission of one request.  set / gb: the idle entries it reuses (-1: a new
// one is allocated).  evict_*: idle entries to free first so that the new
// ones fit.  The reused entries are never among them (freeing the block a
// request is about to render into would leave it without memory).
// fits = false: the request waits, and nothing is to be evicted.
struct Plan {
    int set = -1, gb = -1;
    std::vector<int> evict_sets, evict_gbs;
    uint64_t need = 0;  // bytes of the new allocations
    bool fits = false;
};

// `used` counts every live entry, busy or idle.
inline Plan plan(const std::vector<Set>& sets, const std::vector<Gb>& gbs, uint64_t used, uint64_t budget,
                 const Want& w)
{
    Plan p;
    for (int i = 0; i < (int)sets.size(); ++i) {
        const Set& s = sets[i];
        if (s.v && !s.busy && s.scene == w.scene && s.k == w.k && s.n == w.n && s.h == w.h) {
            p.set = i;
            break;
        }
    }
    for (int i = 0; i < (int)gbs.size(); ++i) {
        const Gb& g = gbs[i];
        if (g.mem && !g.busy && g.bytes >= w.gb_bytes && g.bytes <= 2 * w.gb_bytes) {
            p.gb = i;
            break;
        }
    }
    p.need = (p.set < 0 ? w.set_bytes : 0) + (p.gb < 0 ? w.gb_bytes : 0);
    if (used + p.need <= budget) {
        p.fits = true;
        return p;
    }
    uint64_t idle = 0;
    for (int i = 0; i < (int)sets.size(); ++i)
        if (sets[i].v && !sets[i].busy && i != p.set) idle += sets[i].bytes;
    for (int i = 0; i < (int)gbs.size(); ++i)
        if (gbs[i].mem && !gbs[i].busy && i != p.gb) idle += gbs[i].bytes;
    if (used - idle + p.need > budget) return p;
    uint64_t u = used;
    for (int i = 0; i < (int)sets.size() && u + p.need > budget; ++i)
        if (sets[i].v && !sets[i].busy && i != p.set) {
            p.evict_sets.push_back(i);
            u -= sets[i].bytes;
        }
    for (int i = 0; i < (int)gbs.size() && u + p.need > budget; ++i)
        if (gbs[i].mem && !gbs[i].busy && i != p.gb) {
            p.evict_gbs.push_back(i);
            u -= gbs[i].bytes;
        }
    p.fits = true;
    return p;
}

}  // namespace pool
}  // namespace vplg
