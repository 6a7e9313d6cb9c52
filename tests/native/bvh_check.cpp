// Host check of the BVH builder (bvh_build.cpp) on a triangle soup read from a
// file: the structure of the device arrays and the conservativeness of the
// node boxes.  Usage: bvh_check <file> <segments>; the file holds int32 T and
// then T x 9 float32 vertices.  Exit status 0 when every check holds.
//
// Checked:
// * the leaves' ranges partition [0, T) and the records' ids are a
//   permutation of the triangles; every record holds its triangle's vertices;
// * every inner node is reached once from the root, inner nodes = leaves - 1
//   (or one root over a single leaf), depth <= kMaxDepth - 1;
// * each child box holds its leaf's vertices, or both child boxes of its
//   inner node;
// * the node's split word: axis in {0, 1, 2}, child 0's box centre not above
//   child 1's along it, and the key of (c0.hi + c1.lo) / 2 in the high bits;
// * for random segments, every triangle that the segment crosses (an FP64
//   test, brute force over all triangles) lies in a leaf that an FP64 slab
//   walk of the tree reaches.
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <random>
#include <string>
#include <vector>

#include "vplg_impl.h"

namespace vplg {
bool build_bvh(const float* xyz, int T, std::vector<float4>& out_nodes, std::vector<float4>& out_tris, int* n_leaves,
               int* max_depth, std::string& err);
}
using namespace vplg;

static int fails = 0;
#define CHECK(c, ...)                                                  \
    do {                                                               \
        if (!(c)) {                                                    \
            if (fails < 20) { printf("FAIL: " __VA_ARGS__); printf("\n"); } \
            ++fails;                                                   \
        }                                                              \
    } while (0)

struct Child {
    double lo[3], hi[3];
    int ref, cnt;
};

static Child child_of(const std::vector<float4>& nodes, int n, int c)
{
    const float4* nd = &nodes[4 * (size_t)n];
    const float4 a = c == 0 ? nd[0] : nd[1];
    Child ch;
    ch.lo[0] = a.x; ch.hi[0] = a.y; ch.lo[1] = a.z; ch.hi[1] = a.w;
    ch.lo[2] = c == 0 ? nd[2].x : nd[2].z;
    ch.hi[2] = c == 0 ? nd[2].y : nd[2].w;
    int ints[4];
    std::memcpy(ints, &nd[3], 16);
    ch.ref = ints[c];
    ch.cnt = c == 0 ? (ints[2] & 0xffff) : (ints[2] >> 16);
    return ch;
}

static bool inside(const Child& b, const double* p)
{
    for (int k = 0; k < 3; ++k)
        if (p[k] < b.lo[k] || p[k] > b.hi[k]) return false;
    return true;
}

// segment p + s (q - p), s in [s0, s1], against a box (FP64 slabs)
static bool seg_box(const double* p, const double* d, double s0, double s1, const Child& b)
{
    for (int k = 0; k < 3; ++k) {
        if (d[k] == 0.0) {
            if (p[k] < b.lo[k] || p[k] > b.hi[k]) return false;
            continue;
        }
        double a = (b.lo[k] - p[k]) / d[k], c = (b.hi[k] - p[k]) / d[k];
        if (a > c) std::swap(a, c);
        s0 = std::max(s0, a);
        s1 = std::min(s1, c);
    }
    return s0 <= s1;
}

// FP64 segment-triangle crossing with parameter in (s0, s1)
static bool seg_tri(const double* p, const double* d, double s0, double s1, const double* v)
{
    const double e1[3] = {v[3] - v[0], v[4] - v[1], v[5] - v[2]};
    const double e2[3] = {v[6] - v[0], v[7] - v[1], v[8] - v[2]};
    const double h[3] = {d[1] * e2[2] - d[2] * e2[1], d[2] * e2[0] - d[0] * e2[2], d[0] * e2[1] - d[1] * e2[0]};
    const double det = e1[0] * h[0] + e1[1] * h[1] + e1[2] * h[2];
    if (det == 0.0) return false;
    const double f = 1.0 / det;
    const double sv[3] = {p[0] - v[0], p[1] - v[1], p[2] - v[2]};
    const double u = f * (sv[0] * h[0] + sv[1] * h[1] + sv[2] * h[2]);
    if (u < 0.0 || u > 1.0) return false;
    const double q[3] = {sv[1] * e1[2] - sv[2] * e1[1], sv[2] * e1[0] - sv[0] * e1[2], sv[0] * e1[1] - sv[1] * e1[0]};
    const double w = f * (d[0] * q[0] + d[1] * q[1] + d[2] * q[2]);
    if (w < 0.0 || u + w > 1.0) return false;
    const double s = f * (e2[0] * q[0] + e2[1] * q[1] + e2[2] * q[2]);
    return s > s0 && s < s1;
}

int main(int argc, char** argv)
{
    if (argc < 3) { printf("usage: bvh_check <file> <segments>\n"); return 2; }
    FILE* f = std::fopen(argv[1], "rb");
    if (!f) { perror(argv[1]); return 2; }
    int T = 0;
    if (std::fread(&T, 4, 1, f) != 1 || T <= 0) return 2;
    std::vector<float> xyz(9 * (size_t)T);
    if (std::fread(xyz.data(), 4, xyz.size(), f) != xyz.size()) return 2;
    std::fclose(f);
    const int n_seg = std::atoi(argv[2]);

    std::vector<float4> nodes, tris;
    int n_leaves = 0, max_depth = 0;
    std::string err;
    if (!build_bvh(xyz.data(), T, nodes, tris, &n_leaves, &max_depth, err)) { printf("FAIL: build: %s\n", err.c_str()); return 1; }
    const int nn = (int)nodes.size() / 4;
    const float4* plane2 = tris.data() + 2 * (size_t)kTriStride * T;

    // records: ids a permutation, vertices those of the triangle
    std::vector<int> seen(T, 0), leaf_of(T, -1);
    for (int i = 0; i < T; ++i) {
        int id;
        std::memcpy(&id, &plane2[kTriStride * (size_t)i].w, 4);
        CHECK(id >= 0 && id < T, "record %d has id %d", i, id);
        if (id < 0 || id >= T) continue;
        seen[id]++;
        for (int v = 0; v < 3; ++v) {
            const float4 r = plane2[kTriStride * (size_t)i + v];
            const float* p = &xyz[9 * (size_t)id + 3 * v];
            CHECK(r.x == p[0] && r.y == p[1] && r.z == p[2], "record %d vertex %d differs from triangle %d", i, v, id);
        }
    }
    for (int t = 0; t < T; ++t) CHECK(seen[t] == 1, "triangle %d has %d records", t, seen[t]);

    // walk the tree: each inner node once, leaves partition [0, T), boxes nest
    std::vector<int> reached(nn, 0);
    std::vector<int> covered(T, 0);
    int leaves = 0, depth_max = 0;
    struct Item { int node, depth; };
    std::vector<Item> st = {{0, 0}};
    while (!st.empty()) {
        const Item it = st.back();
        st.pop_back();
        CHECK(it.node >= 0 && it.node < nn, "node index %d out of range", it.node);
        if (it.node < 0 || it.node >= nn) continue;
        reached[it.node]++;
        const Child c[2] = {child_of(nodes, it.node, 0), child_of(nodes, it.node, 1)};
        int split;
        std::memcpy(&split, &nodes[4 * (size_t)it.node + 3].w, 4);
        const int axis = split & 3;
        CHECK(axis <= 2, "node %d axis %d", it.node, axis);
        const bool one_leaf = nn == 1 && c[0].cnt > 0 && c[0].ref == c[1].ref && c[0].cnt == c[1].cnt;
        if (axis <= 2 && !one_leaf) {
            CHECK(c[0].lo[axis] + c[0].hi[axis] <= c[1].lo[axis] + c[1].hi[axis], "node %d children out of order", it.node);
            const float m = 0.5f * ((float)c[0].hi[axis] + (float)c[1].lo[axis]);
            int b;
            std::memcpy(&b, &m, 4);
            CHECK((split & ~3) == ((b ^ ((b >> 31) & 0x7fffffff)) & ~3), "node %d split key", it.node);
        }
        for (int k = 0; k < 2; ++k) {
            if (one_leaf && k == 1) break;
            if (c[k].cnt > 0) {
                leaves++;
                depth_max = std::max(depth_max, it.depth + 1);
                for (int i = c[k].ref; i < c[k].ref + c[k].cnt; ++i) {
                    CHECK(i >= 0 && i < T, "leaf range past the records");
                    if (i < 0 || i >= T) continue;
                    covered[i]++;
                    for (int v = 0; v < 3; ++v) {
                        const float4 r = plane2[kTriStride * (size_t)i + v];
                        const double p[3] = {r.x, r.y, r.z};
                        CHECK(inside(c[k], p), "node %d child %d box misses a vertex of record %d", it.node, k, i);
                    }
                    leaf_of[i] = it.node * 2 + k;
                }
            } else {
                const Child g0 = child_of(nodes, c[k].ref, 0), g1 = child_of(nodes, c[k].ref, 1);
                for (int q = 0; q < 3; ++q)
                    CHECK(c[k].lo[q] <= std::min(g0.lo[q], g1.lo[q]) && c[k].hi[q] >= std::max(g0.hi[q], g1.hi[q]),
                          "node %d child %d box does not hold its children", it.node, k);
                st.push_back({c[k].ref, it.depth + 1});
            }
        }
    }
    for (int n = 0; n < nn; ++n) CHECK(reached[n] == 1, "node %d reached %d times", n, reached[n]);
    for (int i = 0; i < T; ++i) CHECK(covered[i] == 1, "record %d in %d leaves", i, covered[i]);
    CHECK(leaves == n_leaves, "leaves %d, builder says %d", leaves, n_leaves);
    CHECK(nn == std::max(1, leaves - 1), "%d inner nodes for %d leaves", nn, leaves);
    // leaf depth in edges from the root (a lone leaf is its own root: depth 0)
    const bool lone = nn == 1 && leaves == 1;
    CHECK((lone ? 0 : depth_max) == max_depth, "depth %d, builder says %d", lone ? 0 : depth_max, max_depth);
    CHECK(max_depth <= kMaxDepth - 1, "depth %d over the stack", max_depth);

    // conservativeness: every crossed triangle is in a reached leaf
    double lo[3] = {1e30, 1e30, 1e30}, hi[3] = {-1e30, -1e30, -1e30};
    for (size_t i = 0; i < xyz.size(); ++i) {
        lo[i % 3] = std::min(lo[i % 3], (double)xyz[i]);
        hi[i % 3] = std::max(hi[i % 3], (double)xyz[i]);
    }
    std::mt19937_64 rng(12345);
    std::uniform_real_distribution<double> U(0.0, 1.0);
    std::vector<double> vd(9 * (size_t)T);
    for (size_t i = 0; i < vd.size(); ++i) vd[i] = xyz[i];
    std::vector<char> hit_leaf(2 * (size_t)nn);
    long long crossings = 0;
    for (int s = 0; s < n_seg; ++s) {
        double p[3], q[3], d[3];
        for (int k = 0; k < 3; ++k) {
            p[k] = lo[k] + (hi[k] - lo[k]) * U(rng);
            q[k] = lo[k] + (hi[k] - lo[k]) * U(rng);
            d[k] = q[k] - p[k];
        }
        // a third of the segments start on a triangle, as shadow rays do
        if (s % 3 == 0) {
            const int t = (int)(U(rng) * T) % T;
            const double a = U(rng), b = U(rng) * (1.0 - a);
            for (int k = 0; k < 3; ++k) {
                const double* v = &vd[9 * (size_t)t];
                p[k] = v[k] + a * (v[3 + k] - v[k]) + b * (v[6 + k] - v[k]);
                d[k] = q[k] - p[k];
            }
        }
        std::fill(hit_leaf.begin(), hit_leaf.end(), 0);
        std::vector<int> walk = {0};
        while (!walk.empty()) {
            const int n = walk.back();
            walk.pop_back();
            for (int k = 0; k < 2; ++k) {
                const Child c = child_of(nodes, n, k);
                if (!seg_box(p, d, 0.0, 1.0, c)) continue;
                if (c.cnt > 0) hit_leaf[2 * (size_t)n + k] = 1;
                else walk.push_back(c.ref);
            }
        }
        for (int i = 0; i < T; ++i) {
            int id;
            std::memcpy(&id, &plane2[kTriStride * (size_t)i].w, 4);
            if (!seg_tri(p, d, 1e-9, 1.0 - 1e-9, &vd[9 * (size_t)id])) continue;
            crossings++;
            CHECK(hit_leaf[leaf_of[i]], "segment %d crosses triangle %d but the walk misses its leaf", s, id);
        }
    }
    printf("T=%d nodes=%d leaves=%d depth=%d segments=%d crossings=%lld fails=%d\n", T, nn, leaves, max_depth, n_seg,
           crossings, fails);
    return fails == 0 ? 0 : 1;
}
