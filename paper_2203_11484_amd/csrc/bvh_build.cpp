// Host binned-SAH BVH builder for the device layout described in vplg_impl.h.
//
// 32 bins per axis on the centroid bounds, surface-area cost with a unit
// traversal cost and unit triangle cost, leaves of at most 8 triangles.  The
// depth stays below kMaxDepth: deep subtrees fall back to median splits,
// which halve the primitive count per level.  The inner structure is then
// improved by insertion-based optimisation (Bittner, Hapala and Havran,
// "Fast Insertion-Based Optimization of Bounding Volume Hierarchies", 2013)
// over the fixed leaves.  Child boxes are padded outward so that FP32 and
// FP64 slab tests stay conservative.
#include <algorithm>
#include <cfloat>
#include <cmath>
#include <cstring>
#include <functional>
#include <queue>
#include <string>
#include <utility>
#include <vector>

#include "vplg_impl.h"

namespace vplg {

namespace {

constexpr int kBins = 32;
constexpr int kLeafMax = 8;

struct Box {
    float lo[3] = {FLT_MAX, FLT_MAX, FLT_MAX};
    float hi[3] = {-FLT_MAX, -FLT_MAX, -FLT_MAX};
    void grow(const float* p)
    {
        for (int k = 0; k < 3; ++k) {
            lo[k] = std::min(lo[k], p[k]);
            hi[k] = std::max(hi[k], p[k]);
        }
    }
    void grow(const Box& b)
    {
        for (int k = 0; k < 3; ++k) {
            lo[k] = std::min(lo[k], b.lo[k]);
            hi[k] = std::max(hi[k], b.hi[k]);
        }
    }
    bool empty() const { return lo[0] > hi[0]; }
    double area() const
    {
        if (empty()) return 0.0;
        double x = hi[0] - lo[0], y = hi[1] - lo[1], z = hi[2] - lo[2];
        return 2.0 * (x * y + y * z + z * x);
    }
};

struct BNode {
    Box box;
    int left = -1, right = -1;
    int first = 0, count = 0;  // leaf iff count > 0
    int depth = 0;
    int axis = 0;  // split axis of an inner node: the left child's box centre is the lower along it
    int parent = -1;
};

struct Builder {
    const float* xyz;
    std::vector<Box> pbox;
    std::vector<float> cen;  // 3 per primitive
    std::vector<int> idx;
    std::vector<BNode> nodes;
    int sah_depth_limit = 32;
    int max_depth = 0;
    int n_leaves = 0;

    int make_leaf(int begin, int end, const Box& b, int depth)
    {
        BNode n;
        n.box = b;
        n.first = begin;
        n.count = end - begin;
        n.depth = depth;
        nodes.push_back(n);
        max_depth = std::max(max_depth, depth);
        n_leaves++;
        return (int)nodes.size() - 1;
    }

    int build(int begin, int end, int depth)
    {
        Box b, cb;
        for (int i = begin; i < end; ++i) {
            b.grow(pbox[idx[i]]);
            cb.grow(&cen[3 * idx[i]]);
        }
        int n = end - begin;
        if (n <= 2) return make_leaf(begin, end, b, depth);
        int axis = 0;
        float ext[3] = {cb.hi[0] - cb.lo[0], cb.hi[1] - cb.lo[1], cb.hi[2] - cb.lo[2]};
        if (ext[1] > ext[axis]) axis = 1;
        if (ext[2] > ext[axis]) axis = 2;
        int mid = -1;
        int split_axis = axis;
        if (ext[axis] <= 0.f) {
            if (n <= kLeafMax) return make_leaf(begin, end, b, depth);
            mid = begin + n / 2;  // identical centroids: split the list
        } else if (depth >= sah_depth_limit) {
            mid = begin + n / 2;
            std::nth_element(idx.begin() + begin, idx.begin() + mid, idx.begin() + end, [&](int a, int c) {
                float ka = cen[3 * a + axis], kc = cen[3 * c + axis];
                return ka < kc || (ka == kc && a < c);
            });
        } else {
            double best_cost = DBL_MAX;
            int best_axis = -1, best_split = -1;
            for (int ax = 0; ax < 3; ++ax) {
                if (ext[ax] <= 0.f) continue;
                Box bins[kBins];
                int cnt[kBins] = {0};
                float scale = (float)kBins / ext[ax];
                for (int i = begin; i < end; ++i) {
                    int p = idx[i];
                    int bi = std::min(kBins - 1, (int)((cen[3 * p + ax] - cb.lo[ax]) * scale));
                    cnt[bi]++;
                    bins[bi].grow(pbox[p]);
                }
                double rarea[kBins];
                int rcnt[kBins];
                Box acc;
                int c = 0;
                for (int i = kBins - 1; i > 0; --i) {
                    acc.grow(bins[i]);
                    c += cnt[i];
                    rarea[i] = acc.area();
                    rcnt[i] = c;
                }
                Box lacc;
                int lc = 0;
                for (int i = 0; i < kBins - 1; ++i) {
                    lacc.grow(bins[i]);
                    lc += cnt[i];
                    if (lc == 0 || rcnt[i + 1] == 0) continue;
                    double cost = lacc.area() * lc + rarea[i + 1] * rcnt[i + 1];
                    if (cost < best_cost) {
                        best_cost = cost;
                        best_axis = ax;
                        best_split = i;
                    }
                }
            }
            double leaf_cost = (double)n;
            double split_cost = best_axis >= 0 ? 1.0 + best_cost / std::max(b.area(), 1e-30) : DBL_MAX;
            if (n <= kLeafMax && split_cost >= leaf_cost) return make_leaf(begin, end, b, depth);
            if (best_axis >= 0) {
                float scale = (float)kBins / ext[best_axis];
                float lo = cb.lo[best_axis];
                auto it = std::partition(idx.begin() + begin, idx.begin() + end, [&](int p) {
                    int bi = std::min(kBins - 1, (int)((cen[3 * p + best_axis] - lo) * scale));
                    return bi <= best_split;
                });
                mid = (int)(it - idx.begin());
                split_axis = best_axis;
            }
            if (mid <= begin || mid >= end) {
                mid = begin + n / 2;
                split_axis = axis;
                std::nth_element(idx.begin() + begin, idx.begin() + mid, idx.begin() + end, [&](int a, int c) {
                    float ka = cen[3 * a + axis], kc = cen[3 * c + axis];
                    return ka < kc || (ka == kc && a < c);
                });
            }
        }
        BNode node;
        node.box = b;
        node.depth = depth;
        node.axis = split_axis;
        nodes.push_back(node);
        int me = (int)nodes.size() - 1;
        int l = build(begin, mid, depth + 1);
        int r = build(mid, end, depth + 1);
        nodes[me].left = l;
        nodes[me].right = r;
        return me;
    }
};

// Insertion-based optimisation of a built tree.  With the leaves fixed, the
// SAH cost of the tree differs only by the summed surface area of its inner
// nodes.  Each pass takes the tenth of the inner nodes that are largest
// against their children (area^3 / (mean child area x smaller child area)),
// removes each such node N with its parent (N's sibling takes the parent's
// place), and inserts N's two children again, larger first, each as the
// sibling of the node where it adds the least area to the tree, the two freed
// nodes becoming their new parents.  That node comes from a best-first search
// from the root: placing a box b beside node X costs area(X u b) plus what b
// adds to the areas of X's ancestors, and the search stops once that added
// area plus area(b) reaches the best cost found.  Passes stop when the total
// inner area has not fallen by 0.1% for five passes; the best tree within the
// depth limit is kept.  Children are then ordered along the axis of their
// largest centre separation (the lower centre first).
struct Optimizer {
    std::vector<BNode>& n;
    int root;

    double area(int x) const { return n[x].box.area(); }
    static double area_union(const Box& a, const Box& b)
    {
        Box u = a;
        u.grow(b);
        return u.area();
    }
    void refit_up(int x)
    {
        for (; x >= 0; x = n[x].parent) {
            Box b = n[n[x].left].box;
            b.grow(n[n[x].right].box);
            n[x].box = b;
        }
    }
    void replace_child(int p, int oldc, int newc)
    {
        n[newc].parent = p;
        if (p < 0) { root = newc; return; }
        if (n[p].left == oldc) n[p].left = newc;
        else n[p].right = newc;
    }
    int best_sibling(const Box& b) const
    {
        const double ab = b.area();
        double best = DBL_MAX;
        int bx = root;
        using Entry = std::pair<double, int>;  // (area added above the node, node)
        std::priority_queue<Entry, std::vector<Entry>, std::greater<Entry>> pq;
        pq.push({0.0, root});
        while (!pq.empty()) {
            const Entry e = pq.top();
            pq.pop();
            if (e.first + ab >= best) break;
            const BNode& x = n[e.second];
            const double direct = area_union(x.box, b);
            const double cost = e.first + direct;
            if (cost < best) { best = cost; bx = e.second; }
            if (x.count == 0) {
                const double below = cost - x.box.area();
                if (below + ab < best) {
                    pq.push({below, x.left});
                    pq.push({below, x.right});
                }
            }
        }
        return bx;
    }
    void insert(int l, int f)
    {
        const int x = best_sibling(n[l].box);
        const int xp = n[x].parent;
        n[f].count = 0;
        n[f].left = x;
        n[f].right = l;
        replace_child(xp, x, f);
        n[x].parent = f;
        n[l].parent = f;
        refit_up(f);
    }
    // N: an inner node picked at the start of the pass; earlier moves of the
    // pass may have made it the root, which has no parent to remove
    void reinsert(int N)
    {
        if (N == root) return;
        const int P = n[N].parent;
        const int S = n[P].left == N ? n[P].right : n[P].left;
        const int G = n[P].parent;
        replace_child(G, P, S);
        refit_up(G);
        int L = n[N].left, R = n[N].right;
        if (area(L) < area(R)) std::swap(L, R);
        insert(L, N);
        insert(R, P);
    }
    double inner_area() const
    {
        double s = 0.0;
        for (const BNode& b : n)
            if (b.count == 0) s += b.box.area();
        return s;
    }
    int depth() const
    {
        int md = 0;
        std::vector<std::pair<int, int>> st = {{root, 0}};
        while (!st.empty()) {
            const std::pair<int, int> e = st.back();
            st.pop_back();
            md = std::max(md, e.second);
            if (n[e.first].count == 0) {
                st.push_back({n[e.first].left, e.second + 1});
                st.push_back({n[e.first].right, e.second + 1});
            }
        }
        return md;
    }
    void run(int depth_limit)
    {
        for (int i = 0; i < (int)n.size(); ++i)
            if (n[i].count == 0) n[n[i].left].parent = n[n[i].right].parent = i;
        n[root].parent = -1;
        double best = inner_area();
        std::vector<BNode> keep = n;
        int keep_root = root;
        int stall = 0;
        std::vector<std::pair<double, int>> m;
        for (int pass = 0; pass < 100 && stall < 5; ++pass) {
            m.clear();
            for (int i = 0; i < (int)n.size(); ++i) {
                if (n[i].count > 0 || i == root) continue;
                const double a = area(i), a0 = area(n[i].left), a1 = area(n[i].right);
                const double mean = std::max(0.5 * (a0 + a1), 1e-30), small = std::max(std::min(a0, a1), 1e-30);
                m.push_back({a * a * a / (mean * small), i});
            }
            if (m.empty()) break;
            const size_t k = std::max<size_t>(1, m.size() / 10);
            std::partial_sort(m.begin(), m.begin() + k, m.end(), std::greater<std::pair<double, int>>());
            for (size_t i = 0; i < k; ++i) reinsert(m[i].second);
            const double c = inner_area();
            const bool fits = depth() <= depth_limit;
            if (fits && c < best * (1.0 - 1e-3)) stall = 0;
            else ++stall;
            if (fits && c < best) {
                best = c;
                keep = n;
                keep_root = root;
            }
        }
        n = keep;
        root = keep_root;
        for (BNode& b : n) {
            if (b.count > 0) continue;
            const Box& l = n[b.left].box;
            const Box& r = n[b.right].box;
            int axis = 0;
            float sep = -1.f;
            for (int k = 0; k < 3; ++k) {
                const float d = std::fabs((r.lo[k] + r.hi[k]) - (l.lo[k] + l.hi[k]));
                if (d > sep) { sep = d; axis = k; }
            }
            if (l.lo[axis] + l.hi[axis] > r.lo[axis] + r.hi[axis]) std::swap(b.left, b.right);
            b.axis = axis;
        }
    }
};

inline float pad_down(float v, float pad) { return std::nextafter(v - pad, -FLT_MAX); }
inline float pad_up(float v, float pad) { return std::nextafter(v + pad, FLT_MAX); }

}  // namespace

// Build the BVH of T triangles (xyz: [T][3][3]).  Outputs the device node
// array (4 float4 per node) and the leaf-ordered triangle array (3 float4
// per triangle).  Returns false with a message on failure.
bool build_bvh(const float* xyz, int T, std::vector<float4>& out_nodes, std::vector<float4>& out_tris, int* n_leaves,
               int* max_depth, std::string& err)
{
    Builder B;
    B.xyz = xyz;
    B.pbox.resize(T);
    B.cen.resize(3 * (size_t)T);
    B.idx.resize(T);
    float maxabs = 0.f;
    for (int t = 0; t < T; ++t) {
        for (int v = 0; v < 3; ++v) {
            const float* p = xyz + 9 * (size_t)t + 3 * v;
            B.pbox[t].grow(p);
            for (int k = 0; k < 3; ++k) maxabs = std::max(maxabs, std::fabs(p[k]));
        }
        for (int k = 0; k < 3; ++k) B.cen[3 * (size_t)t + k] = 0.5f * (B.pbox[t].lo[k] + B.pbox[t].hi[k]);
        B.idx[t] = t;
    }
    // median levels needed below the SAH levels: ceil(log2(T / leaf)) + 1
    int med = 1;
    while ((1ll << med) * kLeafMax < (long long)T) med++;
    B.sah_depth_limit = std::max(8, kMaxDepth - 2 - med);
    B.nodes.reserve(2 * (size_t)T);
    int root = B.build(0, T, 0);
    if (B.max_depth > kMaxDepth - 1) {
        err = "BVH deeper than the traversal stack";
        return false;
    }
    if (B.nodes[root].count == 0) {
        Optimizer opt{B.nodes, root};
        opt.run(kMaxDepth - 1);
        root = opt.root;
        B.max_depth = opt.depth();
    }
    // flatten: device nodes are the inner build nodes; a leaf-only tree gets
    // an inner root whose two children are that one leaf, so that every
    // device node has two present children
    std::vector<int> dev_of(B.nodes.size(), -1);
    std::vector<int> order;
    if (B.nodes[root].count > 0) {
        order.push_back(-1);
    } else {
        std::vector<int> stack = {root};
        while (!stack.empty()) {
            int n = stack.back();
            stack.pop_back();
            dev_of[n] = (int)order.size();
            order.push_back(n);
            const BNode& bn = B.nodes[n];
            if (B.nodes[bn.right].count == 0) stack.push_back(bn.right);
            if (B.nodes[bn.left].count == 0) stack.push_back(bn.left);
        }
    }
    float pad = 1e-6f * std::max(maxabs, 1.0f);
    out_nodes.assign(4 * order.size(), make_float4(0, 0, 0, 0));
    auto child = [&](int c, float* lo, float* hi, int* ref, int* cnt) {
        // leaf counts share one word: the builder keeps them far below 2^16
        const BNode& n = B.nodes[c];
        for (int k = 0; k < 3; ++k) {
            lo[k] = pad_down(n.box.lo[k], pad);
            hi[k] = pad_up(n.box.hi[k], pad);
        }
        if (n.count > 0) { *ref = n.first; *cnt = n.count; }
        else { *ref = dev_of[c]; *cnt = 0; }
    };
    for (size_t i = 0; i < order.size(); ++i) {
        int l, r;
        int axis = 0;
        if (order[i] < 0) { l = root; r = root; }
        else { l = B.nodes[order[i]].left; r = B.nodes[order[i]].right; axis = B.nodes[order[i]].axis; }
        float lo0[3], hi0[3], lo1[3], hi1[3];
        int c0, c1, k0, k1;
        child(l, lo0, hi0, &c0, &k0);
        child(r, lo1, hi1, &c1, &k1);
        float4* o = &out_nodes[4 * i];
        o[0] = make_float4(lo0[0], hi0[0], lo0[1], hi0[1]);
        o[1] = make_float4(lo1[0], hi1[0], lo1[1], hi1[1]);
        o[2] = make_float4(lo0[2], hi0[2], lo1[2], hi1[2]);
        // the plane between the children along the split axis, as an
        // order-preserving integer key (its two low bits carry the axis)
        const float split = 0.5f * (hi0[axis] + lo1[axis]);
        int sbits;
        std::memcpy(&sbits, &split, sizeof sbits);
        const int skey = sbits ^ ((sbits >> 31) & 0x7fffffff);
        float f[4];
        int ints[4] = {c0, c1, k0 | (k1 << 16), (skey & ~3) | axis};
        std::memcpy(f, ints, sizeof f);
        o[3] = make_float4(f[0], f[1], f[2], f[3]);
    }
    // three planes of T records: plane k holds each vertex permuted as
    // (v[kx], v[ky], v[kz]) for dominant ray axis kz = k (kx, ky the next
    // axes in cyclic order); plane 2 is the identity order and the only one
    // with the normal
    out_tris.assign(3 * kTriStride * (size_t)T, make_float4(0.f, 0.f, 0.f, 0.f));
    float4* plane2 = out_tris.data() + 2 * kTriStride * (size_t)T;
    for (int i = 0; i < T; ++i) {
        int t = B.idx[i];
        const float* p = xyz + 9 * (size_t)t;
        float idf;
        std::memcpy(&idf, &t, sizeof idf);
        double e1[3] = {(double)p[3] - p[0], (double)p[4] - p[1], (double)p[5] - p[2]};
        double e2[3] = {(double)p[6] - p[0], (double)p[7] - p[1], (double)p[8] - p[2]};
        double n[3] = {e1[1] * e2[2] - e1[2] * e2[1], e1[2] * e2[0] - e1[0] * e2[2], e1[0] * e2[1] - e1[1] * e2[0]};
        float nf[3] = {(float)n[0], (float)n[1], (float)n[2]};
        double cut = kParallelTau * kParallelTau *
                     ((double)nf[0] * nf[0] + (double)nf[1] * nf[1] + (double)nf[2] * nf[2]);
        if (!((float)cut > 0.f)) cut = HUGE_VAL;  // degenerate: never hit
        plane2[kTriStride * i] = make_float4(p[0], p[1], p[2], idf);
        plane2[kTriStride * i + 1] = make_float4(p[3], p[4], p[5], (float)cut);
        plane2[kTriStride * i + 2] = make_float4(p[6], p[7], p[8], 0.f);
        plane2[kTriStride * i + 3] = make_float4(nf[0], nf[1], nf[2], 0.f);
        for (int kz = 0; kz < 2; ++kz) {
            const int kx = kz + 1, ky = (kz + 2) % 3;
            float4* r = out_tris.data() + kTriStride * ((size_t)kz * T + i);
            r[0] = make_float4(p[kx], p[ky], p[kz], idf);
            r[1] = make_float4(p[3 + kx], p[3 + ky], p[3 + kz], (float)cut);
            r[2] = make_float4(p[6 + kx], p[6 + ky], p[6 + kz], 0.f);
        }
    }
    *n_leaves = B.n_leaves;
    *max_depth = B.max_depth;
    return true;
}

}  // namespace vplg
