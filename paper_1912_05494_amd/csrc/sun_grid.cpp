// sun_grid.cpp -- host builder of the sun-aligned candidate grid (see
// sun_grid.hpp).  Padding: projections are widened by 2e-5 of the scene
// extent, far beyond the rounding of the device's FP32 projection of a ray
// origin and of the triangle test's acceptance at edges, so every triangle
// that the test can report as crossed is listed in the ray's cell.  A
// triangle is listed in the cells its widened projection meets (not every
// cell of its bounding box), which halves the lists of slanted triangles.
#include "sun_grid.hpp"

#include <algorithm>
#include <cmath>
#include <cstring>

namespace sdm {

SunGrid build_sun_grid(const TriDev *tris, int32_t nt, const int32_t *mat_type, const float sun[3],
                       double extent)
{
    SunGrid g;
    const double sl = std::sqrt((double)sun[0] * sun[0] + (double)sun[1] * sun[1] + (double)sun[2] * sun[2]);
    if (nt <= 0 || !(sl > 0.0) || !std::isfinite(sl)) return g;
    const double s[3] = {sun[0] / sl, sun[1] / sl, sun[2] / sl};
    // basis of the plane perpendicular to the sun: e1 = h x s normalised, e2 = s x e1,
    // h the coordinate axis least aligned with s
    int k = 0;
    for (int a = 1; a < 3; ++a)
        if (std::fabs(s[a]) < std::fabs(s[k])) k = a;
    double h[3] = {0, 0, 0};
    h[k] = 1.0;
    double e1[3] = {h[1] * s[2] - h[2] * s[1], h[2] * s[0] - h[0] * s[2], h[0] * s[1] - h[1] * s[0]};
    const double l1 = std::sqrt(e1[0] * e1[0] + e1[1] * e1[1] + e1[2] * e1[2]);
    for (double &x : e1) x /= l1;
    const double e2[3] = {s[1] * e1[2] - s[2] * e1[1], s[2] * e1[0] - s[0] * e1[2], s[0] * e1[1] - s[1] * e1[0]};
    for (int a = 0; a < 3; ++a) {
        g.e1[a] = (float)e1[a];
        g.e2[a] = (float)e2[a];
    }
    // the device projects with these float vectors and measures depth along
    // the scene's own (float) sun direction
    const double marg = 2e-5 * extent + 1e-30;
    g.marg = (float)marg;
    std::vector<double> amin(nt), amax(nt), bmin(nt), bmax(nt), smin(nt), smax(nt);
    std::vector<double> pa(3 * (size_t)nt), pb(3 * (size_t)nt);   // projected vertices
    double U0 = INFINITY, U1 = -INFINITY, V0 = INFINITY, V1 = -INFINITY;
    for (int32_t i = 0; i < nt; ++i) {
        const float4 v[3] = {tris[i].a, tris[i].b, tris[i].c};
        double a0 = INFINITY, a1 = -INFINITY, b0 = INFINITY, b1 = -INFINITY, s0 = INFINITY, s1 = -INFINITY;
        for (int q = 0; q < 3; ++q) {
            const float4 &p = v[q];
            const double a = p.x * (double)g.e1[0] + p.y * (double)g.e1[1] + p.z * (double)g.e1[2];
            const double b = p.x * (double)g.e2[0] + p.y * (double)g.e2[1] + p.z * (double)g.e2[2];
            pa[3 * (size_t)i + q] = a;
            pb[3 * (size_t)i + q] = b;
            const double d = p.x * (double)sun[0] + p.y * (double)sun[1] + p.z * (double)sun[2];
            a0 = std::min(a0, a); a1 = std::max(a1, a);
            b0 = std::min(b0, b); b1 = std::max(b1, b);
            s0 = std::min(s0, d); s1 = std::max(s1, d);
        }
        amin[i] = a0 - marg; amax[i] = a1 + marg;
        bmin[i] = b0 - marg; bmax[i] = b1 + marg;
        smin[i] = s0; smax[i] = s1;
        U0 = std::min(U0, amin[i]); U1 = std::max(U1, amax[i]);
        V0 = std::min(V0, bmin[i]); V1 = std::max(V1, bmax[i]);
    }
    if (!std::isfinite(U0 + U1 + V0 + V1)) return g;
    // about sixteen cells per triangle, square cells, at most 4096 per side:
    // a wave's walk lasts as long as its longest list, and finer cells
    // shorten the lists (shadow walk on the nave: 4.99 ms at four cells per
    // triangle, 4.69 at eight, 4.62 at sixteen)
    const double du = U1 - U0, dv = V1 - V0;
    const double cell = std::sqrt(du * dv / (16.0 * nt));
    g.nx = (int32_t)std::min(4096.0, std::max(1.0, std::ceil(du / std::max(cell, 1e-30))));
    g.ny = (int32_t)std::min(4096.0, std::max(1.0, std::ceil(dv / std::max(cell, 1e-30))));
    g.u0 = (float)U0;
    g.v0 = (float)V0;
    g.idu = (float)(g.nx / du);
    g.idv = (float)(g.ny / dv);
    const size_t ncell = (size_t)g.nx * g.ny;
    auto cx = [&](double a) { return (int32_t)std::min<double>(g.nx - 1, std::max(0.0, std::floor((a - g.u0) * g.idu))); };
    auto cy = [&](double b) { return (int32_t)std::min<double>(g.ny - 1, std::max(0.0, std::floor((b - g.v0) * g.idv))); };
    // Does triangle i's projection, widened by marg, meet cell (x, y)?  The
    // cell is enlarged by marg on every side and tested against the
    // triangle's edge lines (separating axes; the coordinate axes are
    // already covered by the bounding-box range of cells visited).  Cells
    // are taken a little larger than the device's float cell bounds (1e-4
    // of a cell), so rounding in the cell index never drops a candidate.
    const double cw = 1.0 / g.idu, ch = 1.0 / g.idv;
    auto overlaps = [&](int32_t i, int32_t x, int32_t y) {
        const double ex = marg + 1e-4 * cw, ey = marg + 1e-4 * ch;
        const double r0 = g.u0 + x * cw - ex, r1 = g.u0 + (x + 1) * cw + ex;
        const double s0 = g.v0 + y * ch - ey, s1 = g.v0 + (y + 1) * ch + ey;
        const double *A = &pa[3 * (size_t)i], *B = &pb[3 * (size_t)i];
        for (int e = 0; e < 3; ++e) {
            const int f = (e + 1) % 3, o = (e + 2) % 3;
            const double nx = B[f] - B[e], ny = A[e] - A[f];   // edge normal
            const double len = std::sqrt(nx * nx + ny * ny);
            if (!(len > 0.0)) continue;                        // degenerate edge: no axis
            const double c = nx * A[e] + ny * B[e];
            const double side = nx * A[o] + ny * B[o] - c;     // where the third vertex lies
            if (std::fabs(side) <= 1e-12 * len * (std::fabs(c) / len + 1.0)) continue;   // flat triangle
            // the rectangle corner farthest toward the triangle's side
            const double best = (side > 0 ? std::max(nx * r0, nx * r1) + std::max(ny * s0, ny * s1)
                                          : std::min(nx * r0, nx * r1) + std::min(ny * s0, ny * s1)) - c;
            if (side > 0 ? best < -marg * len : best > marg * len) return false;
        }
        return true;
    };
    std::vector<int64_t> cnt(ncell + 1, 0);
    int64_t total = 0;
    for (int32_t i = 0; i < nt; ++i) {
        const int32_t x0 = cx(amin[i]), x1 = cx(amax[i]), y0 = cy(bmin[i]), y1 = cy(bmax[i]);
        for (int32_t y = y0; y <= y1; ++y)
            for (int32_t x = x0; x <= x1; ++x)
                if (overlaps(i, x, y)) {
                    ++cnt[(size_t)y * g.nx + x];
                    ++total;
                }
        if (total > 96ll * nt + 1024) return g;   // projections too large for a grid: keep the BVH
    }
    // expected candidates of a ray: cells weighted by how often rays fall in them,
    // taken proportional to their list lengths
    double w = 0.0, w2 = 0.0;
    for (size_t c = 0; c < ncell; ++c) {
        w += (double)cnt[c];
        w2 += (double)cnt[c] * cnt[c];
    }
    if (w > 0.0 && w2 / w > 96.0) return g;
    g.start.assign(ncell + 1, 0);
    for (size_t c = 0; c < ncell; ++c) g.start[c + 1] = g.start[c] + (int32_t)cnt[c];
    g.cand.resize((size_t)total);
    std::vector<int32_t> fill(g.start.begin(), g.start.end() - 1);
    std::vector<int32_t> order(nt);
    for (int32_t i = 0; i < nt; ++i) order[i] = i;
    // filling in order of smallest depth keeps every cell's list sorted by it
    std::stable_sort(order.begin(), order.end(), [&](int32_t p, int32_t q) { return smin[p] < smin[q]; });
    for (int32_t i : order) {
        const int32_t x0 = cx(amin[i]), x1 = cx(amax[i]), y0 = cy(bmin[i]), y1 = cy(bmax[i]);
        // largest depth rounded up, so that "below origin depth - marg" is a safe skip
        const float sm = std::nextafter((float)smax[i], INFINITY);
        int32_t mi;
        std::memcpy(&mi, &tris[i].b.w, 4);
        // type in the low two bits, material index above: the walk reports a
        // pane's material without loading its triangle
        const int32_t mt = mat_type[mi] | mi << 2;
        float fl, fm;
        std::memcpy(&fl, &i, 4);
        std::memcpy(&fm, &mt, 4);
        GridCand gc;
        gc.a = make_float4(tris[i].a.x, tris[i].a.y, tris[i].a.z, fl);
        gc.b = make_float4(tris[i].b.x, tris[i].b.y, tris[i].b.z, sm);
        gc.c = make_float4(tris[i].c.x, tris[i].c.y, tris[i].c.z, fm);
        for (int32_t y = y0; y <= y1; ++y)
            for (int32_t x = x0; x <= x1; ++x)
                if (overlaps(i, x, y)) g.cand[fill[(size_t)y * g.nx + x]++] = gc;
    }
    g.use = true;
    return g;
}

}  // namespace sdm
