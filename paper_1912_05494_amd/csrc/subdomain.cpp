// subdomain.cpp -- geometric sub-domains (Sec. 5): the scene's bounds cut into
// a grid of cells, each with its own wide BVH (the builder of bvh_build.cpp)
// over the triangles whose bounding boxes overlap the cell.
#include "subdomain.hpp"

#include <algorithm>
#include <cmath>

#include "bvh_build.hpp"

namespace sdm {

SubdomainBuild build_subdomains(const float *pos, int32_t nv, const int32_t *idx, int32_t nt,
                                const std::vector<TriDev> &leaf_tris, const std::vector<int32_t> &o2l,
                                const int32_t n[3], const double lo[3], const double hi[3])
{
    SubdomainBuild out;
    double diag = 0.0;
    for (int a = 0; a < 3; ++a) diag += (hi[a] - lo[a]) * (hi[a] - lo[a]);
    diag = std::sqrt(diag);
    const double margin = 1e-5 * diag + 1e-20;
    // cell faces along each axis, shared by neighbouring cells
    std::vector<float> edge[3];
    for (int a = 0; a < 3; ++a) {
        const double g0 = lo[a] - margin, g1 = hi[a] + margin;
        edge[a].resize(n[a] + 1);
        for (int k = 0; k <= n[a]; ++k) edge[a][k] = (float)(g0 + (g1 - g0) * k / n[a]);
        edge[a][n[a]] = (float)g1;
        out.lo[a] = edge[a][0];
        out.size[a] = (float)((g1 - g0) / n[a]);
    }
    const int64_t n_cells = (int64_t)n[0] * n[1] * n[2];
    std::vector<std::vector<int32_t>> lists((size_t)n_cells);
    for (int32_t t = 0; t < nt; ++t) {
        float tl[3], th[3];
        for (int a = 0; a < 3; ++a) {
            tl[a] = INFINITY;
            th[a] = -INFINITY;
        }
        for (int c = 0; c < 3; ++c)
            for (int a = 0; a < 3; ++a) {
                const float x = pos[3 * (size_t)idx[3 * (size_t)t + c] + a];
                tl[a] = std::min(tl[a], x);
                th[a] = std::max(th[a], x);
            }
        int k0[3], k1[3];
        for (int a = 0; a < 3; ++a) {
            // cells k with edge[k] - margin <= th and edge[k + 1] + margin >= tl
            k0[a] = 0;
            while (k0[a] < n[a] - 1 && (double)edge[a][k0[a] + 1] + margin < (double)tl[a]) ++k0[a];
            k1[a] = n[a] - 1;
            while (k1[a] > 0 && (double)edge[a][k1[a]] - margin > (double)th[a]) --k1[a];
        }
        for (int z = k0[2]; z <= k1[2]; ++z)
            for (int y = k0[1]; y <= k1[1]; ++y)
                for (int x = k0[0]; x <= k1[0]; ++x) lists[((size_t)z * n[1] + y) * n[0] + x].push_back(t);
    }
    std::vector<int32_t> sub;
    for (int z = 0; z < n[2]; ++z)
        for (int y = 0; y < n[1]; ++y)
            for (int x = 0; x < n[0]; ++x) {
                const std::vector<int32_t> &L = lists[((size_t)z * n[1] + y) * n[0] + x];
                CellDev c;
                const int k[3] = {x, y, z};
                for (int a = 0; a < 3; ++a) {
                    c.lo[a] = edge[a][k[a]];
                    c.hi[a] = edge[a][k[a] + 1];
                }
                c.node_base = (int32_t)out.nodes.size();
                c.tri_base = (int32_t)out.tris.size();
                c.n_nodes = 0;
                c.n_tris = (int32_t)L.size();
                if (!L.empty()) {
                    sub.resize(3 * L.size());
                    for (size_t i = 0; i < L.size(); ++i)
                        for (int q = 0; q < 3; ++q) sub[3 * i + q] = idx[3 * (size_t)L[i] + q];
                    BvhResult b = build_bvh(pos, nv, sub.data(), (int32_t)L.size());
                    out.ok = out.ok && b.ok;
                    c.n_nodes = (int32_t)b.nodes.size();
                    out.nodes.insert(out.nodes.end(), b.nodes.begin(), b.nodes.end());
                    for (size_t l = 0; l < b.order.size(); ++l) {
                        const int32_t t = L[b.order[l]];
                        out.tris.push_back(leaf_tris[o2l[t]]);
                        out.leaf.push_back(o2l[t]);
                    }
                    out.stack = std::max(out.stack, b.stack);
                }
                out.cells.push_back(c);
            }
    return out;
}

}  // namespace sdm
