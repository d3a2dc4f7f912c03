// sdm_dev.hpp -- device-side building blocks of the spectral wavefront tracer
// (gfx950, wave64).  Templated on the geometry/shading precision R (float for
// production, double for the validation build of the same kernels).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "sdm_types.hpp"

namespace sdm {

// ---------------------------------------------------------------------------
// Counter-based random numbers: Philox4x32-10 (Salmon, Moraes, Dror, Shaw,
// SC'11).  Each round multiplies words 0 and 2 by the round constants, mixes
// the high halves with words 1 and 3 and the key, and bumps the key by the
// Weyl increments.
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint4 philox10(uint4 c, uint2 k)
{
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint32_t lo0 = 0xD2511F53u * c.x, hi0 = __umulhi(0xD2511F53u, c.x);
        const uint32_t lo1 = 0xCD9E8D57u * c.z, hi1 = __umulhi(0xCD9E8D57u, c.z);
        c = make_uint4(hi1 ^ c.y ^ k.x, lo1, hi0 ^ c.w ^ k.y, lo0);
        k.x += 0x9E3779B9u;
        k.y += 0xBB67AE85u;
    }
    return c;
}

// Uniform in [0, 1) from the top 24 bits: exact in float and double.
template <class R>
__device__ __forceinline__ R u01(uint32_t x)
{
    return R(x >> 8) * R(1.0 / 16777216.0);
}

// Draws of one path vertex: counter (pixel, sample, (vertex+1) << 16 | call,
// job word), key = seed.  Vertex -1 is the camera.  The wavelength is not in
// the counter: every wavelength of a (pixel, sample) sees the same numbers,
// which is what lets one ray carry a whole spectral band.
__device__ __forceinline__ uint4 vertex_draws(uint64_t seed, uint32_t job_word, uint32_t pixel,
                                              uint32_t sample, int vertex, uint32_t call)
{
    return philox10(make_uint4(pixel, sample, ((uint32_t)(vertex + 1) << 16) | call, job_word),
                    make_uint2((uint32_t)seed, (uint32_t)(seed >> 32)));
}

// ---------------------------------------------------------------------------
// Small vector type
// ---------------------------------------------------------------------------
template <class R>
struct V3 {
    R x, y, z;
};
template <class R> __device__ __forceinline__ V3<R> mk(R x, R y, R z) { return V3<R>{x, y, z}; }
template <class R> __device__ __forceinline__ V3<R> operator+(V3<R> a, V3<R> b) { return {a.x + b.x, a.y + b.y, a.z + b.z}; }
template <class R> __device__ __forceinline__ V3<R> operator-(V3<R> a, V3<R> b) { return {a.x - b.x, a.y - b.y, a.z - b.z}; }
template <class R> __device__ __forceinline__ V3<R> operator*(R s, V3<R> a) { return {s * a.x, s * a.y, s * a.z}; }
template <class R> __device__ __forceinline__ R dot(V3<R> a, V3<R> b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
template <class R> __device__ __forceinline__ V3<R> cross(V3<R> a, V3<R> b)
{
    return {a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x};
}
template <class R> __device__ __forceinline__ V3<R> normalize(V3<R> a)
{
    R l = sqrt(dot(a, a));
    return l > R(0) ? V3<R>{a.x / l, a.y / l, a.z / l} : a;
}
template <class R> __device__ __forceinline__ V3<R> from4(float4 f) { return {R(f.x), R(f.y), R(f.z)}; }

// Tangent basis about unit n from the fixed axis h = (1, 2, 3) / sqrt(14):
// t1 = normalize(h x n), t2 = n x t1.  Continuous for every normal but +-h,
// so vertical and axis-aligned faces get the same basis whatever the sign of
// the rounding residue in their normal's zero components.
template <class R>
__device__ __forceinline__ void onb(V3<R> n, V3<R> &t1, V3<R> &t2)
{
    const V3<R> h = {R(0.2672612419124244), R(0.5345224838248488), R(0.8017837257372732)};
    t1 = normalize(cross(h, n));
    t2 = cross(n, t1);
}

// Cosine-weighted direction about n: uniform disk point (r = sqrt(u1),
// phi = 2 pi u2) lifted to the hemisphere.
template <class R>
__device__ __forceinline__ V3<R> cosine_dir(V3<R> n, R u1, R u2)
{
    V3<R> t1, t2;
    onb(n, t1, t2);
    const R r = sqrt(u1), lz = sqrt(R(1) - u1);
    R s, c;
    // FP32: the angle 2 pi u2 as sincospi(2 u2), which needs no reduction of
    // large arguments (the general sincos carries one, and its registers)
    if constexpr (sizeof(R) == 4) sincospif(R(2) * u2, &s, &c);
    else sincos(R(6.283185307179586) * u2, &s, &c);
    return (r * c) * t1 + (r * s) * t2 + lz * n;
}

// Four consecutive values of a 16-byte aligned per-wavelength row, moved with
// 16-byte loads and stores (one for float, two for double).
template <class R>
struct Vec4 {
    R v[4];
};
template <class R>
__device__ __forceinline__ Vec4<R> row_load4(const R *p)
{
    Vec4<R> r;
    if constexpr (sizeof(R) == 4) {
        const float4 a = *reinterpret_cast<const float4 *>(p);
        r.v[0] = a.x; r.v[1] = a.y; r.v[2] = a.z; r.v[3] = a.w;
    } else {
        const double2 a = reinterpret_cast<const double2 *>(p)[0], b = reinterpret_cast<const double2 *>(p)[1];
        r.v[0] = a.x; r.v[1] = a.y; r.v[2] = b.x; r.v[3] = b.y;
    }
    return r;
}
template <class R>
__device__ __forceinline__ void row_store4(R *p, const Vec4<R> &r)
{
    if constexpr (sizeof(R) == 4) {
        *reinterpret_cast<float4 *>(p) = make_float4(r.v[0], r.v[1], r.v[2], r.v[3]);
    } else {
        reinterpret_cast<double2 *>(p)[0] = make_double2(r.v[0], r.v[1]);
        reinterpret_cast<double2 *>(p)[1] = make_double2(r.v[2], r.v[3]);
    }
}

// ---------------------------------------------------------------------------
// Glass: thin slab with Fresnel interfaces for n~ = n + ik (eq. (1)).
// ---------------------------------------------------------------------------
// Principal square root of a complex number (re >= 0), written to avoid
// cancellation in the smaller component.
template <class R>
__device__ __forceinline__ void csqrt_p(R zr, R zi, R &sr, R &si)
{
    const R m = hypot(zr, zi);
    if (m == R(0)) { sr = R(0); si = R(0); return; }
    if (zr >= R(0)) {
        sr = sqrt(R(0.5) * (m + zr));
        si = zi / (R(2) * sr);
    } else {
        R t = sqrt(R(0.5) * (m - zr));
        si = copysign(t, zi);
        sr = fabs(zi) / (R(2) * t);
    }
}

// Interface reflectances air -> n + ik at incidence cosine c, s and p.
template <class R>
__device__ __forceinline__ void fresnel_sp(R c, R n, R k, R &Rs, R &Rp)
{
    c = fmin(fmax(c, R(0)), R(1));
    const R s2 = R(1) - c * c;
    const R a = n * n - k * k, b = R(2) * n * k;     // n~^2
    const R m = a * a + b * b;
    // cos(theta_t) = sqrt(1 - s2 / n~^2) on the principal branch
    R cr, ci;
    csqrt_p(R(1) - s2 * a / m, s2 * b / m, cr, ci);
    const R x = n * cr - k * ci, y = n * ci + k * cr; // n~ cos(theta_t)
    Rs = ((c - x) * (c - x) + y * y) / ((c + x) * (c + x) + y * y);
    const R px = n * c, py = k * c;                  // n~ cos(theta_i)
    Rp = ((px - cr) * (px - cr) + (py - ci) * (py - ci)) /
         ((px + cr) * (px + cr) + (py + ci) * (py + ci));
}

// a / b for the slab optics: times the hardware reciprocal in FP32 (within
// about one unit in the last place, against a correctly rounded division's
// half; the FP32 kernels are held to the FP64 oracle by tolerance), a
// division in FP64.
template <class R>
__device__ __forceinline__ R slab_div(R a, R b)
{
    if constexpr (sizeof(R) == 4) return a * __builtin_amdgcn_rcpf(b);
    else return a / b;
}

template <class R>
__device__ __forceinline__ void slab_pol(R r, R tau, R &Rr, R &Tt)
{
    if (r >= R(1)) { Rr = R(1); Tt = R(0); return; }
    // R = r + (1-r)^2 r tau^2 / (1 - r^2 tau^2), T = (1-r)^2 tau / (1 - r^2 tau^2),
    // with one division for both
    const R q = R(1) - r;
    const R rt = r * tau;
    const R inv = slab_div(R(1), R(1) - rt * rt);
    const R qqt = q * q * tau;
    Rr = r + qqt * rt * inv;
    Tt = qqt * inv;
}

// Slab reflectance/transmittance: Fresnel per polarisation at both faces,
// Beer-Lambert attenuation exp(-alpha d / cos(theta_t)) with alpha = 4 pi k /
// lambda + alpha_tint and the real Snell angle, incoherent multiple
// reflections summed in closed form, s and p averaged.
template <class R>
__device__ __forceinline__ void slab_RT(R c, R lambda_nm, R d_mm, R n, R k, R tint, R &Rout, R &Tout)
{
    c = fmin(fmax(c, R(0)), R(1));
    const R st = slab_div(sqrt(fmax(R(1) - c * c, R(0))), n);
    const R ct2 = R(1) - st * st;
    const R ct = ct2 > R(0) ? sqrt(ct2) : R(0);
    R Rs, Rp;
    if (sizeof(R) == 4 && k < R(2.5e-4)) {
        // FP32: the complex index changes the reflectances by O(k^2), at most
        // the unit roundoff here, so the real-index form (on the Snell cosine
        // the path length uses anyway) gives the same values; both ratios
        // (c - n ct) / (c + n ct) and (n c - ct) / (n c + ct) share one division
        const R nc = n * c, nct = n * ct;
        const R a = c + nct, b = nc + ct;
        const R inv = slab_div(R(1), a * b);
        const R rs = (c - nct) * b * inv, rp = (nc - ct) * a * inv;
        Rs = rs * rs;
        Rp = rp * rp;
    } else {
        fresnel_sp(c, n, k, Rs, Rp);
    }
    // alpha d / ct with alpha = 4 pi k / lambda + tint (lambda in mm):
    // (4 pi 1e6 k + tint lambda_nm) d / (lambda_nm ct), one division
    const R num = (R(12566370.614359172) * k + tint * lambda_nm) * d_mm;
    const R tau = (num == R(0)) ? R(1) : (ct > R(0) ? exp(-slab_div(num, lambda_nm * ct)) : R(0));
    R R1, T1, R2, T2;
    slab_pol(Rs, tau, R1, T1);
    slab_pol(Rp, tau, R2, T2);
    Rout = R(0.5) * (R1 + R2);
    Tout = R(0.5) * (T1 + T2);
}

// ---------------------------------------------------------------------------
// Ray-triangle tests: two-sided, edges inclusive.
// ---------------------------------------------------------------------------
// Moeller-Trumbore (1997), the FP64 test (the same arithmetic as a plain
// double-precision reference).
template <class R>
__device__ __forceinline__ bool tri_hit(V3<R> o, V3<R> d, V3<R> p0, V3<R> p1, V3<R> p2, R &t, R &u, R &v)
{
    const V3<R> e1 = p1 - p0, e2 = p2 - p0;
    const V3<R> pv = cross(d, e2);
    const R det = dot(e1, pv);
    if (det == R(0)) return false;
    const R inv = R(1) / det;
    const V3<R> sv = o - p0;
    u = dot(sv, pv) * inv;
    if (u < R(0) || u > R(1)) return false;
    const V3<R> qv = cross(sv, e1);
    v = dot(d, qv) * inv;
    if (v < R(0) || u + v > R(1)) return false;
    t = dot(e2, qv) * inv;
    return true;
}

// Watertight test for FP32 (Woop, Benthin and Wald, "Watertight
// Ray/Triangle Intersection", JCGT 2013).  The ray is sheared so that it
// runs along +z through the origin: kz is the axis where |d| is largest and
// (kx, ky) = (kz + 1, kz + 2) mod 3, and a point p - o maps to (p[kx] - sx
// p[kz], p[ky] - sy p[kz], sz p[kz]) with (sx, sy, sz) = (d[kx], d[ky], 1) /
// d[kz].  The published test swaps kx and ky when d[kz] < 0 to keep the
// winding; that swap negates U, V, W, det and T exactly (each is a sum of
// products of the swapped coordinates, and rounding is symmetric in sign), so
// without it the accepted rays and t, u, v are the same.  A vertex maps to the
// same floats in every triangle that holds it, and each edge function a.x b.y
// - a.y b.x is evaluated without fused multiply-adds, so the triangle on the
// other side of a shared edge computes exactly its negation: a ray is never
// rejected by both (no crack between neighbours), and a ray on the edge
// (value 0) is accepted by both, the closest-hit tie rule then picking one.
// Rounding is monotone, so near a shared vertex the signs are those of an
// exact point and one triangle of the fan accepts.
//
// The test reads vertices in the ray's frame, (p[kx], p[ky], p[kz]): the
// traversal kernels read them so from a copy of the triangles rotated by kz
// (rot_frame, applied once per scene), which spares the per-lane selection
// of the three coordinates of each vertex; o is the ray origin in that frame.
template <class R>
struct Shear {
    R sx, sy, sz;
    uint32_t kz;
    V3<R> o;
};

// p in the frame of axis kz: (p[kz + 1], p[kz + 2], p[kz]), indices mod 3.
template <class R>
__device__ __forceinline__ V3<R> rot_frame(V3<R> p, uint32_t kz)
{
    return kz == 0u ? V3<R>{p.y, p.z, p.x} : (kz == 1u ? V3<R>{p.z, p.x, p.y} : V3<R>{p.x, p.y, p.z});
}

template <class R>
__device__ __forceinline__ Shear<R> make_shear(V3<R> o, V3<R> d)
{
    const R ax = fabs(d.x), ay = fabs(d.y), az = fabs(d.z);
    Shear<R> s;
    s.kz = (ax >= ay && ax >= az) ? 0u : (ay >= az ? 1u : 2u);
    const V3<R> dr = rot_frame(d, s.kz);
    s.sz = R(1) / dr.z;
    s.sx = dr.x * s.sz;
    s.sy = dr.y * s.sz;
    s.o = rot_frame(o, s.kz);
    return s;
}

// a.x b.y - a.y b.x with both products rounded separately.
__device__ __forceinline__ float edge_fn(float ax, float ay, float bx, float by)
{
#pragma clang fp contract(off)
    return ax * by - ay * bx;
}

// p0, p1, p2 in the ray's frame (see rot_frame).
template <class R>
__device__ __forceinline__ bool tri_hit_wt(const Shear<R> &sh, V3<R> p0, V3<R> p1, V3<R> p2, R &t, R &u, R &v)
{
    static_assert(sizeof(R) == 4, "the watertight form is the FP32 test");
    const V3<R> a = p0 - sh.o, b = p1 - sh.o, c = p2 - sh.o;
    const R ax = a.x - sh.sx * a.z, ay = a.y - sh.sy * a.z;
    const R bx = b.x - sh.sx * b.z, by = b.y - sh.sy * b.z;
    const R cx = c.x - sh.sx * c.z, cy = c.y - sh.sy * c.z;
    // scaled barycentrics: U weighs p0 (edge p1 p2), V p1, W p2
    const R U = edge_fn(cx, cy, bx, by);
    const R V = edge_fn(ax, ay, cx, cy);
    const R W = edge_fn(bx, by, ax, ay);
    if ((U < R(0) || V < R(0) || W < R(0)) && (U > R(0) || V > R(0) || W > R(0))) return false;
    const R det = U + V + W;
    if (det == R(0)) return false;
    const R T = U * (sh.sz * a.z) + V * (sh.sz * b.z) + W * (sh.sz * c.z);
    const R sg = det < R(0) ? R(-1) : R(1), ia = R(1) / fabs(det);
    u = sg * V * ia;
    v = sg * W * ia;
    t = sg * T * ia;
    return true;
}

// Inverse direction for the slab tests.  FP32 takes the hardware reciprocal
// (about one ulp): a slab distance then moves by about 1e-7 of itself, far
// inside the box padding, and hits are decided by the triangle test alone.
template <class R>
__device__ __forceinline__ V3<R> safe_inv(V3<R> d)
{
    const R tiny = sizeof(R) == 4 ? R(1e-20) : R(1e-200);
    auto f = [&](R x) -> R {
        const R y = fabs(x) < tiny ? (x < R(0) ? -tiny : tiny) : x;
        if constexpr (sizeof(R) == 4) return __builtin_amdgcn_rcpf(y);
        else return R(1) / y;
    };
    return V3<R>{f(d.x), f(d.y), f(d.z)};
}

// ---------------------------------------------------------------------------
// Wave-level compaction: one atomic per wave per queue.
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint32_t lane_id() { return __lane_id(); }

// Mask of the wave's active lanes whose pred is set (the vote on the bool
// itself, without widening it to an integer first).
__device__ __forceinline__ uint64_t wave_ballot(bool pred) { return __builtin_amdgcn_ballot_w64(pred); }

// All lanes of the wave must call this together.  Returns the slot of each
// lane with pred set (undefined for the others).
__device__ __forceinline__ uint32_t wave_reserve(bool pred, uint32_t *counter)
{
    const uint64_t m = __ballot(pred);
    const uint32_t lane = lane_id();
    const uint32_t before = (uint32_t)__popcll(m & ((1ull << lane) - 1ull));
    uint32_t base = 0;
    if (m) {
        const int leader = __ffsll((unsigned long long)m) - 1;
        if ((int)lane == leader) base = atomicAdd(counter, (uint32_t)__popcll(m));
        base = __shfl(base, leader);
    }
    return base + before;
}

}  // namespace sdm
