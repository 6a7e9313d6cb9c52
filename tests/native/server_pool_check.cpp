// Host check of the render server's pool bookkeeping (server_pool.h): a FIFO
// admission loop over request mixes, with requests finishing in random order,
// asserts after every admission that
//   * the entries a request reuses are live, and none of them was evicted,
//   * an evicted entry was idle and is not held by any running request,
//   * pooled bytes equal the sum of live entries and stay within the budget,
//   * a request that fits the budget alone is always admitted eventually.
// Usage: server_pool_check random <schedules>
//        server_pool_check mix <schedules>   (stdin: "budget inflight" then
//        one "scene k n gb_bytes set_bytes" line per request)
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <random>
#include <vector>

#include "server_pool.h"

using namespace vplg::pool;

struct Req {
    uint64_t scene;
    int k, n;
    uint64_t gb, set;
};

static int fails = 0;
#define CHECK(c, ...)                                   \
    do {                                                \
        if (!(c)) {                                     \
            if (fails++ < 10) std::printf(__VA_ARGS__); \
            return false;                               \
        }                                               \
    } while (0)

static char g_token;  // stands in for a device allocation

static bool simulate(const std::vector<Req>& reqs, uint64_t budget, int inflight, std::mt19937_64& rng)
{
    std::vector<Set> sets;
    std::vector<Gb> gbs;
    uint64_t used = 0;
    std::vector<int> queue;
    for (int i = 0; i < (int)reqs.size(); ++i) queue.push_back(i);
    struct Run { int req, set, gb; };
    std::vector<Run> running;
    size_t head = 0;
    while (head < queue.size() || !running.empty()) {
        while (head < queue.size() && (int)running.size() < inflight) {
            const Req& r = reqs[queue[head]];
            const Want w{r.scene, r.k, r.n, 0.1, r.gb, r.set};
            const Plan p = plan(sets, gbs, used, budget, w);
            if (!p.fits) {
                CHECK(!running.empty(), "request %d fits alone but is never admitted\n", queue[head]);
                break;
            }
            for (int i : p.evict_sets) {
                CHECK(sets[i].v && !sets[i].busy && i != p.set, "evicted set %d is not an idle other entry\n", i);
                used -= sets[i].bytes;
                sets[i].v = nullptr;
            }
            for (int i : p.evict_gbs) {
                CHECK(gbs[i].mem && !gbs[i].busy && i != p.gb, "evicted block %d is not an idle other entry\n", i);
                used -= gbs[i].bytes;
                gbs[i].mem = nullptr;
            }
            int si = p.set, gi = p.gb;
            CHECK(si < 0 || (sets[si].v && !sets[si].busy), "request %d reuses a freed or held set\n", queue[head]);
            CHECK(gi < 0 || (gbs[gi].mem && !gbs[gi].busy), "request %d reuses a freed or held block\n", queue[head]);
            if (si < 0) {
                Set e;
                e.v = &g_token;
                e.bytes = r.set;
                e.scene = r.scene;
                e.k = r.k;
                e.n = r.n;
                e.h = 0.1;
                used += e.bytes;
                for (int i = 0; i < (int)sets.size(); ++i)
                    if (!sets[i].v) si = i;
                if (si < 0) {
                    sets.push_back(e);
                    si = (int)sets.size() - 1;
                } else {
                    sets[si] = e;
                }
            }
            if (gi < 0) {
                Gb g;
                g.mem = &g_token;
                g.bytes = r.gb;
                used += g.bytes;
                for (int i = 0; i < (int)gbs.size(); ++i)
                    if (!gbs[i].mem) gi = i;
                if (gi < 0) {
                    gbs.push_back(g);
                    gi = (int)gbs.size() - 1;
                } else {
                    gbs[gi] = g;
                }
            }
            sets[si].busy = true;
            gbs[gi].busy = true;
            uint64_t live = 0;
            for (auto& e : sets) live += e.v ? e.bytes : 0;
            for (auto& g : gbs) live += g.mem ? g.bytes : 0;
            CHECK(live == used, "pooled bytes %llu != live bytes %llu\n", (unsigned long long)used,
                  (unsigned long long)live);
            CHECK(used <= budget, "pool %llu over budget %llu\n", (unsigned long long)used,
                  (unsigned long long)budget);
            running.push_back({queue[head], si, gi});
            ++head;
        }
        if (running.empty()) break;
        // a random running request finishes; its entries become idle
        const size_t j = rng() % running.size();
        const Run f = running[j];
        CHECK(sets[f.set].v && sets[f.set].busy && gbs[f.gb].mem && gbs[f.gb].busy,
              "request %d lost its buffers while running\n", f.req);
        sets[f.set].busy = false;
        gbs[f.gb].busy = false;
        running.erase(running.begin() + j);
    }
    CHECK(head == queue.size(), "admission stopped with %zu requests queued\n", queue.size() - head);
    return true;
}

int main(int argc, char** argv)
{
    if (argc < 3) return 2;
    const int schedules = std::atoi(argv[2]);
    int bad = 0;
    if (!std::strcmp(argv[1], "mix")) {
        unsigned long long budget;
        int inflight;
        if (std::scanf("%llu %d", &budget, &inflight) != 2) return 2;
        std::vector<Req> reqs;
        unsigned long long sc, gb, set;
        int k, n;
        while (std::scanf("%llu %d %d %llu %llu", &sc, &k, &n, &gb, &set) == 5) reqs.push_back({sc, k, n, gb, set});
        for (int t = 0; t < schedules; ++t) {
            std::mt19937_64 rng(t);
            bad += !simulate(reqs, budget, inflight, rng);
        }
    } else {
        for (int t = 0; t < schedules; ++t) {
            std::mt19937_64 rng(1000003ull * t + 7);
            // 3 scenes x 3 VPL budgets (set sizes), 4 G-buffer shapes; a budget of 2-4 large requests
            const uint64_t set_mb[3] = {1, 8, 8}, gb_kb[4] = {40, 160, 270, 80};
            std::vector<Req> reqs;
            const int nr = 4 + (int)(rng() % 20);
            for (int i = 0; i < nr; ++i) {
                const int sc = (int)(rng() % 3), kv = (int)(rng() % 3);
                Req r{(uint64_t)sc, 64 << kv, 64 << kv, (gb_kb[rng() % 4] << 10) + (rng() % 4096),
                      (set_mb[sc] << 20) + ((uint64_t)kv << 16) + (rng() % 65536)};
                reqs.push_back(r);
            }
            const uint64_t budget = (uint64_t)(10 + rng() % 24) << 20;
            const int inflight = 1 + (int)(rng() % 8);
            bad += !simulate(reqs, budget, inflight, rng);
        }
    }
    std::printf("%d of %d schedules failed\n", bad, schedules);
    return bad ? 1 : 0;
}
