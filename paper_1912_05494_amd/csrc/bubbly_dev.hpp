// bubbly_dev.hpp -- device code of bubbly glass (air micro-particles in the
// glass body, Sec. 1; volume scattering as the next material feature,
// Sec. 6): the photon walk inside a slab, its frame, the surrogate's lobe and
// the error-table cell of a vertex.
//
// Model: the entry interface uses the complex index n + ik at the wavelength
// (eq. (1)); inside, every direction and every decision (face reflection,
// bubble surfaces) uses the pane's real index n_ref (its index at 560 nm in a
// render), so one walk serves every wavelength that enters and its absorption
// weight is exp(-alpha(lambda) L) over the length L travelled in glass.
// Bubbles: Poisson centres with extinction sigma = rho_b pi <r^2>, acting at
// the collision point with exact sphere optics for the direction (impact
// ratio sqrt(u), glass -> air Fresnel or total reflection at the outer
// surface, else p internal reflections and a deviation 2 (i - r) + p (pi -
// 2 r)); the polarisation label is drawn at entry and afresh at each bubble.
#pragma once
#include <hip/hip_runtime.h>

#include "sdm_dev.hpp"

namespace sdm {

constexpr uint32_t kWalkMaxEvents = 10000;   // then the photon counts as absorbed
constexpr int kWalkMaxInternal = 64;         // internal reflections in one bubble

// Error-table cells: cos(theta) in [0, 1], thickness in [2, 5] mm, bubble
// density in [0, 34] per mm^3, each split evenly; values outside clamp.
constexpr float kErrDLo = 2.0f, kErrDHi = 5.0f, kErrRhoHi = 34.0f;

// Real-index Fresnel reflectance n1 -> n2 at incidence cosine c, polarisation
// pol (0 = s, 1 = p); 1 beyond the critical angle.
template <class R>
__device__ __forceinline__ R fresnel_real(R n1, R n2, R c, int pol)
{
    c = fmin(c, R(1));
    const R st2 = (n1 / n2) * (n1 / n2) * (R(1) - c * c);
    if (st2 >= R(1)) return R(1);
    const R ct = sqrt(R(1) - st2);
    const R r = pol == 0 ? (n1 * c - n2 * ct) / (n1 * c + n2 * ct) : (n2 * c - n1 * ct) / (n2 * c + n1 * ct);
    return r * r;
}

// Draw stream of one walk.  Slab tables: counter (tuple, photon, event,
// 0x5EB10000 | sub).  In a render, at path vertex v of (pixel, sample, job):
// (pixel, sample, 2^31 | v << 23 | event << 5 | sub, job); bit 31 keeps these
// apart from the per-vertex draws, whose third word stays below 2^24.
struct WalkStream {
    uint64_t seed;
    uint32_t c0, c1, c3, vertex;
    bool render;
};

template <class R>
__device__ __forceinline__ void walk_draw(const WalkStream &s, uint32_t event, uint32_t sub, R u[4])
{
    const uint4 c = s.render ? make_uint4(s.c0, s.c1, 0x80000000u | (s.vertex << 23) | (event << 5) | sub, s.c3)
                             : make_uint4(s.c0, s.c1, event, 0x5EB10000u | sub);
    const uint4 x = philox10(c, make_uint2((uint32_t)s.seed, (uint32_t)(s.seed >> 32)));
    u[0] = u01<R>(x.x);
    u[1] = u01<R>(x.y);
    u[2] = u01<R>(x.z);
    u[3] = u01<R>(x.w);
}

template <class R>
struct WalkOut {
    int kind;     // 0 absorbed (event cap), 1 out through the entry face, 2 through the far face
    V3<R> a;      // direction in air, slab frame: x in the plane of incidence, z into the slab
    R L;          // length travelled in glass (mm)
    int bubbles;  // bubbles met (0: the light left unscattered)
};

// The walk after the photon has entered (label pol drawn at entry).
template <class R>
__device__ WalkOut<R> bubbly_walk(const WalkStream &s, R cos_i, R d, R sigma, R n_ref, int pol)
{
    WalkOut<R> out;
    out.kind = 0;
    out.bubbles = 0;
    out.a = {R(0), R(0), R(0)};
    R u[4], v[4];
    const R sin_i = sqrt(fmax(R(1) - cos_i * cos_i, R(0)));
    const R st = sin_i / n_ref;
    V3<R> dir = {st, R(0), sqrt(fmax(R(1) - st * st, R(0)))};
    R z = R(0), L = R(0);
    for (uint32_t e = 1; e <= kWalkMaxEvents; ++e) {
        walk_draw<R>(s, e, 0, u);
        const R sb = dir.z > R(0) ? (d - z) / dir.z : (dir.z < R(0) ? -z / dir.z : R(INFINITY));
        const R l = sigma > R(0) ? -log1p(-u[0]) / sigma : R(INFINITY);
        if (l >= sb) {
            L += sb;
            const bool bottom = dir.z > R(0);
            z = bottom ? d : R(0);
            if (u[1] < fresnel_real<R>(n_ref, R(1), fabs(dir.z), pol)) {
                dir.z = -dir.z;
                continue;
            }
            const R tx = n_ref * dir.x, ty = n_ref * dir.y;
            const R tz = sqrt(fmax(R(1) - tx * tx - ty * ty, R(0)));
            out.kind = bottom ? 2 : 1;
            out.a = {tx, ty, bottom ? tz : -tz};
            out.L = L;
            return out;
        }
        L += l;
        z += l * dir.z;
        ++out.bubbles;
        V3<R> t1, t2;
        onb(dir, t1, t2);
        R sphi, cphi;
        if constexpr (sizeof(R) == 4) sincospif(R(2) * u[3], &sphi, &cphi);
        else sincos(R(6.283185307179586) * u[3], &sphi, &cphi);
        const V3<R> ep = cphi * t1 + sphi * t2;
        uint32_t sub = 1;
        walk_draw<R>(s, e, sub, v);
        pol = v[1] < R(0.5) ? 0 : 1;
        const R sin_b = sqrt(u[2]), cos_b = sqrt(R(1) - u[2]);
        if (v[0] < fresnel_real<R>(n_ref, R(1), cos_b, pol)) {
            const V3<R> nh = (-cos_b) * dir + sin_b * ep;
            dir = dir - (R(2) * dot(dir, nh)) * nh;
        } else {
            const R sr = n_ref * sin_b;
            const R R2 = fresnel_real<R>(R(1), n_ref, sqrt(fmax(R(1) - sr * sr, R(0))), pol);
            int q = 2, p = 0;
            while (p < kWalkMaxInternal) {
                if (q == 4) {
                    walk_draw<R>(s, e, ++sub, v);
                    q = 0;
                }
                if (v[q++] < R2) ++p;
                else break;
            }
            const R ri = asin(fmin(sin_b, R(1))), rr = asin(fmin(sr, R(1)));
            const R D = R(2) * (ri - rr) + R(p) * (R(3.141592653589793) - R(2) * rr);
            R sD, cD;
            if constexpr (sizeof(R) == 4) sincosf(D, &sD, &cD);
            else sincos(D, &sD, &cD);
            dir = cD * dir - sD * ep;
        }
        dir = normalize(dir);
    }
    out.L = L;
    return out;
}

// Slab frame of a hit: z along the face normal on the far side of the ray, x
// along the ray's component in the face (the onb() axis when the ray meets
// the face head-on), y = z x x.
template <class R>
__device__ __forceinline__ V3<R> slab_to_world(V3<R> d, V3<R> ng, V3<R> a)
{
    const R dn = dot(d, ng);
    const V3<R> nz = dn > R(0) ? ng : R(-1) * ng;
    V3<R> ex = d - fabs(dn) * nz, t2;
    const R len = sqrt(dot(ex, ex));
    if (len > R(1e-7)) ex = (R(1) / len) * ex;
    else onb(nz, ex, t2);
    const V3<R> ey = cross(nz, ex);
    return normalize(a.x * ex + a.y * ey + a.z * nz);
}

// Surrogate transmitted direction: d plus a 2-D Gaussian offset of standard
// deviation w per tangent axis (Box-Muller on u1, u2) in the basis onb(d).
template <class R>
__device__ __forceinline__ V3<R> lobe_dir(V3<R> d, R w, R u1, R u2)
{
    V3<R> t1, t2;
    onb(d, t1, t2);
    const R g = sqrt(R(-2) * log1p(-u1));
    R s, c;
    if constexpr (sizeof(R) == 4) sincospif(R(2) * u2, &s, &c);
    else sincos(R(6.283185307179586) * u2, &s, &c);
    return normalize(d + w * ((g * c) * t1 + (g * s) * t2));
}

// Cell of a vertex in the error table [pane][cos][thickness][density].
template <class R>
__device__ __forceinline__ int err_cell(const int dims[3], int pane, R cos_i, R d, R rho)
{
    const int nc = dims[0], nd = dims[1], nr = dims[2];
    int ic = (int)(cos_i * R(nc));
    int id = (int)((d - R(kErrDLo)) / R(kErrDHi - kErrDLo) * R(nd));
    int ir = (int)(rho / R(kErrRhoHi) * R(nr));
    ic = ic < 0 ? 0 : (ic >= nc ? nc - 1 : ic);
    id = id < 0 ? 0 : (id >= nd ? nd - 1 : id);
    ir = ir < 0 ? 0 : (ir >= nr ? nr - 1 : ir);
    return ((pane * nc + ic) * nd + id) * nr + ir;
}

}  // namespace sdm
