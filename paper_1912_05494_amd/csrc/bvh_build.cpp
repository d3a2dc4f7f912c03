// bvh_build.cpp -- host BVH builder: a binary tree by the binned surface-area
// heuristic over the three axes (leaves of at most kLeafMax triangles, depth
// capped), collapsed into 4-wide nodes by opening the largest-area inner
// child until a node has four children, output in breadth-first order (the
// top levels form an index prefix the traversal kernels stage in LDS).
#include <algorithm>
#include <cmath>
#include <cstring>
#include <deque>
#include <limits>
#include <vector>

#include "bvh_build.hpp"

namespace sdm {
namespace {

constexpr int kBins = 16;
constexpr int kLeafMax = 2;

struct Box {
    float lo[3] = {std::numeric_limits<float>::infinity(), std::numeric_limits<float>::infinity(),
                   std::numeric_limits<float>::infinity()};
    float hi[3] = {-std::numeric_limits<float>::infinity(), -std::numeric_limits<float>::infinity(),
                   -std::numeric_limits<float>::infinity()};
    void grow(const Box &b)
    {
        for (int a = 0; a < 3; ++a) {
            lo[a] = std::min(lo[a], b.lo[a]);
            hi[a] = std::max(hi[a], b.hi[a]);
        }
    }
    void grow(const float *p)
    {
        for (int a = 0; a < 3; ++a) {
            lo[a] = std::min(lo[a], p[a]);
            hi[a] = std::max(hi[a], p[a]);
        }
    }
    bool empty() const { return lo[0] > hi[0]; }
    double area() const
    {
        if (empty()) return 0.0;
        double e0 = hi[0] - lo[0], e1 = hi[1] - lo[1], e2 = hi[2] - lo[2];
        return 2.0 * (e0 * e1 + e1 * e2 + e2 * e0);
    }
};

struct TNode {             // temporary tree node
    Box box;
    int32_t left = -1, right = -1;  // children (temporary indices) or -1
    int32_t first = 0, count = 0;   // leaf range in `prims`
    bool leaf() const { return left < 0; }
};

struct Builder {
    const float *pos;
    const int32_t *idx;
    std::vector<Box> tbox;
    std::vector<float> cen;  // [nt*3]
    std::vector<int32_t> prims;
    std::vector<TNode> nodes;
    int max_depth = 0;
    bool too_big = false;   // a depth-capped leaf exceeds kMaxLeafTris

    int32_t make_leaf(const Box &b, int32_t first, int32_t count)
    {
        TNode n;
        n.box = b;
        n.first = first;
        n.count = count;
        nodes.push_back(n);
        return (int32_t)nodes.size() - 1;
    }

    int32_t build(int32_t first, int32_t count, int depth)
    {
        max_depth = std::max(max_depth, depth + 1);
        Box b, cb;
        for (int32_t i = first; i < first + count; ++i) {
            b.grow(tbox[prims[i]]);
            cb.grow(&cen[3 * (size_t)prims[i]]);
        }
        if (count <= kLeafMax) return make_leaf(b, first, count);
        // binned SAH over the three axes
        double best_cost = std::numeric_limits<double>::infinity();
        int best_axis = -1, best_split = -1;
        for (int a = 0; a < 3; ++a) {
            const float ext = cb.hi[a] - cb.lo[a];
            if (!(ext > 0.0f)) continue;
            Box bb[kBins];
            int32_t bc[kBins] = {0};
            const float scale = kBins / ext;
            for (int32_t i = first; i < first + count; ++i) {
                int bin = (int)((cen[3 * (size_t)prims[i] + a] - cb.lo[a]) * scale);
                bin = std::min(std::max(bin, 0), kBins - 1);
                bb[bin].grow(tbox[prims[i]]);
                bc[bin]++;
            }
            Box lb[kBins], rb[kBins];
            int32_t lc[kBins], rc[kBins];
            Box acc;
            int32_t n = 0;
            for (int i = 0; i < kBins; ++i) {
                acc.grow(bb[i]);
                n += bc[i];
                lb[i] = acc;
                lc[i] = n;
            }
            acc = Box();
            n = 0;
            for (int i = kBins - 1; i >= 0; --i) {
                acc.grow(bb[i]);
                n += bc[i];
                rb[i] = acc;
                rc[i] = n;
            }
            for (int s = 0; s < kBins - 1; ++s) {
                if (lc[s] == 0 || rc[s + 1] == 0) continue;
                const double c = lb[s].area() * lc[s] + rb[s + 1].area() * rc[s + 1];
                if (c < best_cost) {
                    best_cost = c;
                    best_axis = a;
                    best_split = s;
                }
            }
        }
        int32_t mid;
        if (best_axis < 0) {
            // all centroids coincide: split by count
            mid = first + count / 2;
        } else {
            const float ext = cb.hi[best_axis] - cb.lo[best_axis];
            const float scale = kBins / ext;
            auto it = std::partition(prims.begin() + first, prims.begin() + first + count,
                                     [&](int32_t p) {
                                         int bin = (int)((cen[3 * (size_t)p + best_axis] -
                                                          cb.lo[best_axis]) * scale);
                                         bin = std::min(std::max(bin, 0), kBins - 1);
                                         return bin <= best_split;
                                     });
            mid = (int32_t)(it - prims.begin());
            if (mid == first || mid == first + count) mid = first + count / 2;
        }
        if (depth + 1 >= kMaxBvhDepth) {
            if (count > kMaxLeafTris) too_big = true;
            return make_leaf(b, first, count);
        }
        TNode n;
        n.box = b;
        nodes.push_back(n);
        const int32_t me = (int32_t)nodes.size() - 1;
        const int32_t l = build(first, mid - first, depth + 1);
        const int32_t r = build(mid, first + count - mid, depth + 1);
        nodes[me].left = l;
        nodes[me].right = r;
        return me;
    }
};

void set_child(BvhNode &g, int which, const Box &b, int32_t entry, float pad_abs)
{
    if (entry == kNoChild || b.empty()) {
        g.lox[which] = g.loy[which] = g.loz[which] = std::numeric_limits<float>::infinity();
        g.hix[which] = g.hiy[which] = g.hiz[which] = -std::numeric_limits<float>::infinity();
        g.child[which] = kNoChild;
        return;
    }
    float lo[3], hi[3];
    for (int a = 0; a < 3; ++a) {
        const float p = pad_abs + 1e-5f * std::max(std::fabs(b.lo[a]), std::fabs(b.hi[a]));
        lo[a] = b.lo[a] - p;
        hi[a] = b.hi[a] + p;
    }
    g.lox[which] = lo[0]; g.loy[which] = lo[1]; g.loz[which] = lo[2];
    g.hix[which] = hi[0]; g.hiy[which] = hi[1]; g.hiz[which] = hi[2];
    g.child[which] = entry;
}

int32_t leaf_entry(const TNode &n) { return -1 - ((n.first << 8) | n.count); }

// Children of the wide node rooted at binary node t: start from its two
// children and open the inner child of largest surface area until there are
// four or only leaves remain.
int collapse(const std::vector<TNode> &nodes, int32_t t, int32_t (&kids)[4])
{
    int nk = 2;
    kids[0] = nodes[t].left;
    kids[1] = nodes[t].right;
    while (nk < 4) {
        int best = -1;
        double best_area = -1.0;
        for (int i = 0; i < nk; ++i) {
            const TNode &c = nodes[kids[i]];
            if (!c.leaf() && c.box.area() > best_area) {
                best_area = c.box.area();
                best = i;
            }
        }
        if (best < 0) break;
        const TNode &c = nodes[kids[best]];
        kids[best] = c.left;
        kids[nk++] = c.right;
    }
    return nk;
}

}  // namespace

BvhResult build_bvh(const float *pos, int32_t nv, const int32_t *idx, int32_t nt)
{
    BvhResult out;
    if (nt <= 0) return out;
    Builder B;
    B.pos = pos;
    B.idx = idx;
    B.tbox.resize(nt);
    B.cen.resize(3 * (size_t)nt);
    B.prims.resize(nt);
    Box scene;
    for (int32_t t = 0; t < nt; ++t) {
        Box b;
        for (int c = 0; c < 3; ++c) b.grow(pos + 3 * (size_t)idx[3 * (size_t)t + c]);
        B.tbox[t] = b;
        for (int a = 0; a < 3; ++a) B.cen[3 * (size_t)t + a] = 0.5f * (b.lo[a] + b.hi[a]);
        B.prims[t] = t;
        scene.grow(b);
    }
    (void)nv;
    B.nodes.reserve(2 * (size_t)nt);
    const int32_t root = B.build(0, nt, 0);
    out.ok = !B.too_big;
    out.order = B.prims;
    double diag = 0.0;
    for (int a = 0; a < 3; ++a) diag += double(scene.hi[a] - scene.lo[a]) * (scene.hi[a] - scene.lo[a]);
    diag = std::sqrt(diag);
    const float pad_abs = (float)(1e-5 * diag) + 1e-30f;

    if (B.nodes[root].leaf()) {   // one leaf: a single node with one child
        BvhNode g;
        std::memset(&g, 0, sizeof(g));
        set_child(g, 0, B.nodes[root].box, leaf_entry(B.nodes[root]), pad_abs);
        for (int w = 1; w < 4; ++w) set_child(g, w, Box(), kNoChild, pad_abs);
        out.nodes.push_back(g);
        out.depth = 2;
        out.stack = 0;
        return out;
    }
    // Breadth-first emission of wide nodes; leaves live in their parent.
    struct Wide {
        int32_t kids[4];
        int nk, level;
    };
    std::vector<Wide> wide;
    std::vector<int32_t> gidx(B.nodes.size(), -1);
    std::deque<std::pair<int32_t, int>> q;
    q.push_back({root, 0});
    gidx[root] = 0;
    int32_t next = 1;
    while (!q.empty()) {
        const auto [t, level] = q.front();
        q.pop_front();
        Wide wn;
        wn.level = level;
        wn.nk = collapse(B.nodes, t, wn.kids);
        for (int i = 0; i < wn.nk; ++i)
            if (!B.nodes[wn.kids[i]].leaf()) {
                gidx[wn.kids[i]] = next++;
                q.push_back({wn.kids[i], level + 1});
            }
        wide.push_back(wn);
    }
    out.nodes.resize(wide.size());
    std::vector<int> need(wide.size(), 0);
    for (size_t i = wide.size(); i-- > 0;) {   // children come after their parent
        const Wide &wn = wide[i];
        BvhNode g;
        std::memset(&g, 0, sizeof(g));
        int deeper = 0;
        for (int w = 0; w < 4; ++w) {
            if (w >= wn.nk) {
                set_child(g, w, Box(), kNoChild, pad_abs);
                continue;
            }
            const TNode &c = B.nodes[wn.kids[w]];
            if (c.leaf()) {
                set_child(g, w, c.box, leaf_entry(c), pad_abs);
            } else {
                set_child(g, w, c.box, gidx[wn.kids[w]], pad_abs);
                deeper = std::max(deeper, need[gidx[wn.kids[w]]]);
            }
        }
        // a walk at this node keeps at most nk - 1 siblings on the stack while
        // it descends into one child
        need[i] = wn.nk - 1 + deeper;
        out.nodes[i] = g;
        out.depth = std::max(out.depth, wn.level + 2);
    }
    out.stack = need[0];
    return out;
}

}  // namespace sdm
