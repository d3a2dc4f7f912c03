// wavefront.hip -- kernels of the spectral wavefront path tracer (gfx950).
//
// A path carries one spectral band (a sub-domain of Sec. 4): all wavelengths
// of a (pixel, sample) draw the same random numbers, and thin-slab glass
// bends no wavelength differently, so they follow one ray until a glass
// vertex sends some wavelengths to reflection and others to transmission;
// then the path forks (wavelengths are still independent, so the image is
// the same as tracing each wavelength alone).
//
// One step of the loop of Sec. 3.1 over a pool of paths:
//   k_trace         closest hit of every path (persistent, lanes refilled)
//   k_shade         a sky record per escaping path, a shadow record per
//                   Lambert vertex (eq. (3)), the cosine bounce, survivors
//                   compacted into the other pool; glass vertices queued
//   k_shade_glass   clear panes: slab R, T per wavelength, reflect or pass,
//                   forks where the wavelengths disagree
//   k_bubbly_eval,  bubbly panes: surrogate network on the matrix cores,
//   k_shade_bubbly  exact walk or surrogate branch
//   k_shadow_trace  any-hit walk of the shadow records toward the sun
//   k_shadow_accum  per wavelength: slab transmittance of the panes crossed
//                   (sun records) or sky radiance (sky records), a pixel's
//                   records summed in registers with lanes over wavelengths,
//                   one FP64 atomic row add per pixel run
// Weights are a scalar per path times per-wavelength factors that exist only
// once the wavelengths' weights differ (kSpectral).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>

#include "../../include/sdm.h"
#include "bubbly_dev.hpp"
#include "mlp_dev.hpp"
#include "sdm_dev.hpp"
#include "surrogate.hpp"
#include "wavefront.hpp"

namespace sdm {

constexpr int kLdsNodes = 160;    // wide-node prefix staged in LDS (20 KB) by the shadow and test kernels
constexpr int kBlock = 256;
constexpr int kTraceBlock = 256;   // threads per block of the closest-hit traversal
constexpr int kTraceNodes = 160;   // wide-node prefix its blocks stage in LDS
constexpr int kShadeBlock = 512;   // threads per block of the shading pass (fewer slot reservations)
constexpr uint32_t kFetch = 256;  // items per group of the traversal work distribution
constexpr int kDescentLanes = 24;  // a closest-hit descent ends when fewer lanes still search
constexpr int32_t kDone = INT_MIN;

// ---------------------------------------------------------------------------
// Explicit global-memory loads (pointers read from structs would otherwise
// be generic and compile to flat loads).
// ---------------------------------------------------------------------------
typedef float f4v __attribute__((ext_vector_type(4)));
__device__ __forceinline__ float4 gld4(const float4 *p)
{
    const f4v v = *(const __attribute__((address_space(1))) f4v *)p;
    return make_float4(v.x, v.y, v.z, v.w);
}
typedef int i4v __attribute__((ext_vector_type(4)));
__device__ __forceinline__ int4 gld4(const int4 *p)
{
    const i4v v = *(const __attribute__((address_space(1))) i4v *)p;
    return make_int4(v.x, v.y, v.z, v.w);
}
template <class T>
__device__ __forceinline__ T gld(const T *p)
{
    return *(const __attribute__((address_space(1))) T *)p;
}

// Records moved as 16-byte words with global loads and stores.
typedef uint32_t u4v __attribute__((ext_vector_type(4)));
template <class T>
__device__ __forceinline__ T rec_load(const T *p)
{
    static_assert(sizeof(T) % 16 == 0, "record size");
    const __attribute__((address_space(1))) u4v *q = (const __attribute__((address_space(1))) u4v *)p;
    u4v t[sizeof(T) / 16];
#pragma unroll
    for (size_t k = 0; k < sizeof(T) / 16; ++k) t[k] = q[k];
    T r;
    __builtin_memcpy(&r, t, sizeof(T));
    return r;
}
template <class T>
__device__ __forceinline__ void rec_store(T *p, const T &r)
{
    static_assert(sizeof(T) % 16 == 0, "record size");
    __attribute__((address_space(1))) u4v *q = (__attribute__((address_space(1))) u4v *)p;
    u4v t[sizeof(T) / 16];
    __builtin_memcpy(t, &r, sizeof(T));
#pragma unroll
    for (size_t k = 0; k < sizeof(T) / 16; ++k) q[k] = t[k];
}

template <class R>
__device__ __forceinline__ void put_path(const Pool<R> &P, uint32_t k, V3<R> o, V3<R> d, int32_t skip, uint32_t pix,
                                         uint32_t smp, uint32_t aux, R g)
{
    PathO<R> a;
    a.x = o.x; a.y = o.y; a.z = o.z; a.skip = skip;
    PathD<R> b;
    b.x = d.x; b.y = d.y; b.z = d.z;
    PathS<R> c;
    c.pix = pix; c.smp = smp; c.aux = aux; c.g = g;
    rec_store(P.o + k, a);
    rec_store(P.d + k, b);
    rec_store(P.s + k, c);
}

// Wavelengths j .. j+3 of a band's row in a wavelength table (rows of ms
// values, ms a multiple of 4).  A band that starts at a multiple of 4 reads
// them with one 16-byte load (two for double); otherwise four loads, each
// clamped to the band's last wavelength so none leaves the row.
typedef double d2v __attribute__((ext_vector_type(2)));
template <class R>
__device__ __forceinline__ Vec4<R> tab4(const R *row, bool aligned, int j, int nb)
{
    Vec4<R> r;
    if (aligned) {
        if constexpr (sizeof(R) == 4) {
            const f4v v = *(const __attribute__((address_space(1))) f4v *)(row + j);
            r.v[0] = v.x; r.v[1] = v.y; r.v[2] = v.z; r.v[3] = v.w;
        } else {
            const __attribute__((address_space(1))) d2v *p = (const __attribute__((address_space(1))) d2v *)(row + j);
            const d2v a = p[0], b = p[1];
            r.v[0] = a.x; r.v[1] = a.y; r.v[2] = b.x; r.v[3] = b.y;
        }
    } else {
#pragma unroll
        for (int q = 0; q < 4; ++q) r.v[q] = gld(row + min(j + q, nb - 1));
    }
    return r;
}

// ---------------------------------------------------------------------------
// Traversal stack: kLdsStack levels per lane in LDS, deeper levels in a
// per-thread global region.  Entries are inner-node indices (>= 0) or leaves
// encoded as -1 - (first << 8 | count).
// ---------------------------------------------------------------------------
typedef __attribute__((address_space(3))) int32_t lds_i32;   // an LDS word (ds_* access)
typedef __attribute__((address_space(1))) int32_t glb_i32;   // a global word (global_* access)
template <int B>   // threads per block
struct StackT {
    lds_i32 *lds;       // [kLdsStack][B]
    glb_i32 *glob;      // [(level - kLdsStack) * gstride + gtid]
    uint32_t gtid, gstride;
    int sp;
    __device__ __forceinline__ void push(int32_t v)
    {
        if (sp < kLdsStack) lds[sp * B + threadIdx.x] = v;
        else glob[(size_t)(sp - kLdsStack) * gstride + gtid] = v;
        ++sp;
    }
    __device__ __forceinline__ int32_t pop()
    {
        --sp;
        return sp < kLdsStack ? lds[sp * B + threadIdx.x] : glob[(size_t)(sp - kLdsStack) * gstride + gtid];
    }
    // Pushes e[m], ..., e[1] (m <= 3), so that e[1] is popped first.  With
    // three free LDS levels the three slots are written whatever m is (slots
    // above the new top are dead), which keeps the lanes of a wave together.
    __device__ __forceinline__ void push_sorted(int m, int32_t e1, int32_t e2, int32_t e3)
    {
        if (sp + 3 <= kLdsStack) {
            lds_i32 *p = lds + sp * B + threadIdx.x;
            p[0] = m == 3 ? e3 : (m == 2 ? e2 : e1);
            p[B] = m == 3 ? e2 : e1;
            p[2 * B] = e1;
            sp += m;
        } else {
            if (m == 3) push(e3);
            if (m >= 2) push(e2);
            if (m >= 1) push(e1);
        }
    }
};

using Stack = StackT<kBlock>;

template <int B = kBlock>
__device__ __forceinline__ StackT<B> make_stack(int32_t *lds_stack, int32_t *gstack)
{
    StackT<B> st;
    st.lds = (lds_i32 *)lds_stack;
    st.glob = (glb_i32 *)gstack;
    st.gtid = blockIdx.x * blockDim.x + threadIdx.x;
    st.gstride = gridDim.x * blockDim.x;
    st.sp = 0;
    return st;
}

// Wide-node fetch.  The first kLdsNodes nodes (the top levels, breadth-first)
// are read from LDS, where the 16-byte word k of node i sits at
// i * 8 + (k ^ (i & 7)): lanes reading the same word of different nodes then
// fall into different bank groups.  The padding word (k = 7) is not read.
// The plane words are read in the ray's octant order: for each axis the near
// planes (lo where the direction is positive, hi where it is negative) and
// the far ones, so the slab test needs no min/max to sort the two distances.
struct WideNode {
    float4 nx, fx, ny, fy, nz, fz;   // near / far planes of the four children per axis
    int32_t c0, c1, c2, c3;   // child entries (separate values: an indexed array would go to scratch)
};

__device__ __forceinline__ int lds_slot(int i, int k) { return i * 8 + (k ^ (i & 7)); }

// kx, ky, kz: byte offsets in the node of the ray's near-plane words (x: 0 or
// 16, y: 32 or 48, z: 64 or 80); the far-plane word is the other of the pair.
__device__ __forceinline__ WideNode load_node(const float4 *lds_nodes, int n_lds, const BvhNode *nodes, int i,
                                              uint32_t kx, uint32_t ky, uint32_t kz)
{
    const uint32_t key[7] = {kx, kx ^ 16u, ky, ky ^ 16u, kz, kz ^ 16u, 96u};
    float4 q[7];
    if (i < n_lds) {
        // byte address of word k: (i * 128 | (i & 7) * 16) ^ k * 16
        const uint32_t a0 = ((uint32_t)i << 7) | (((uint32_t)i & 7u) << 4);
        const char *base = reinterpret_cast<const char *>(lds_nodes);
#pragma unroll
        for (int k = 0; k < 7; ++k) q[k] = *reinterpret_cast<const float4 *>(base + (a0 ^ key[k]));
    } else {
        const char *base = reinterpret_cast<const char *>(nodes);
        const uint32_t a0 = (uint32_t)i << 7;   // node byte offset (nodes < 2^25)
#pragma unroll
        for (int k = 0; k < 7; ++k) q[k] = gld4(reinterpret_cast<const float4 *>(base + (size_t)(a0 | key[k])));
    }
    WideNode n;
    n.nx = q[0]; n.fx = q[1]; n.ny = q[2]; n.fy = q[3]; n.nz = q[4]; n.fz = q[5];
    n.c0 = __float_as_int(q[6].x);
    n.c1 = __float_as_int(q[6].y);
    n.c2 = __float_as_int(q[6].z);
    n.c3 = __float_as_int(q[6].w);
    return n;
}

__device__ __forceinline__ int stage_nodes(float4 *lds_nodes, const SceneDev &sc, int n_max = kLdsNodes)
{
    const int n = min(sc.n_nodes, n_max);
    const float4 *src = reinterpret_cast<const float4 *>(sc.nodes);
    for (int x = threadIdx.x; x < 8 * n; x += blockDim.x) lds_nodes[lds_slot(x >> 3, x & 7)] = gld4(src + x);
    __syncthreads();
    return n;
}

__device__ __forceinline__ float f4get(const float4 &v, int c)
{
    return c == 0 ? v.x : c == 1 ? v.y : c == 2 ? v.z : v.w;
}
__device__ __forceinline__ int32_t child_at(const WideNode &nd, int c)
{
    return c == 0 ? nd.c0 : c == 1 ? nd.c1 : c == 2 ? nd.c2 : nd.c3;
}

template <class R>
struct Ray {
    V3<R> o, d, inv;
    V3<R> oi;            // o * inv, for the fused slab form
    uint32_t kx, ky, kz; // node word offsets of the near planes (see load_node)
    int32_t skip, cur;
    Shear<R> sh;         // ray-space shear of the FP32 triangle test
};

// Triangle test of a ray: watertight in FP32, Moeller-Trumbore in FP64.
// ray_tri takes the vertices in scene coordinates; ray_tri_frame takes them
// as test_tris lists them (in FP32 already in the ray's shear frame).
template <class R>
__device__ __forceinline__ bool ray_tri(const Ray<R> &ry, V3<R> p0, V3<R> p1, V3<R> p2, R &t, R &u, R &v)
{
    if constexpr (sizeof(R) == 4)
        return tri_hit_wt(ry.sh, rot_frame(p0, ry.sh.kz), rot_frame(p1, ry.sh.kz), rot_frame(p2, ry.sh.kz), t, u, v);
    else return tri_hit(ry.o, ry.d, p0, p1, p2, t, u, v);
}

template <class R>
__device__ __forceinline__ bool ray_tri_frame(const Ray<R> &ry, V3<R> p0, V3<R> p1, V3<R> p2, R &t, R &u, R &v)
{
    if constexpr (sizeof(R) == 4) return tri_hit_wt(ry.sh, p0, p1, p2, t, u, v);
    else return tri_hit(ry.o, ry.d, p0, p1, p2, t, u, v);
}

// The triangles a ray's test reads: in FP32 the copy whose vertices are
// rotated into the frame of the ray's dominant axis (same w words, same
// order), in FP64 the scene's own.
template <class R>
__device__ __forceinline__ const TriDev *test_tris(const SceneDev &sc, const Ray<R> &ry)
{
    if constexpr (sizeof(R) == 4) return sc.tris_rot + (size_t)ry.sh.kz * (size_t)sc.rot_n;
    else return sc.tris;
}

template <class R>
__device__ __forceinline__ void set_dir(Ray<R> &ry, V3<R> o, V3<R> d)
{
    ry.o = o;
    ry.d = d;
    ry.inv = safe_inv(d);
    ry.oi = {o.x * ry.inv.x, o.y * ry.inv.y, o.z * ry.inv.z};
    ry.kx = signbit(ry.inv.x) ? 16u : 0u;
    ry.ky = signbit(ry.inv.y) ? 48u : 32u;
    ry.kz = signbit(ry.inv.z) ? 80u : 64u;
    if constexpr (sizeof(R) == 4) ry.sh = make_shear(o, d);
}

// Distance to the plane x = b along one axis.  The fused form b * inv - o *
// inv saves a subtraction per plane; its rounding error, about |o| u in
// distance (u = 2^-24 in FP32), stays far inside the box padding (1e-5 of
// the scene diagonal plus 1e-5 of the box coordinates) when the origin lies
// in the scene's bounds, as it does for rays leaving a surface and for
// pinhole camera rays whose eye lies within the bounds of the scene's
// triangles (the render checks it per job).  Other rays (cameras elsewhere,
// orthographic cameras, test rays) use (b - o) * inv.
template <bool kFused, class R>
__device__ __forceinline__ R slab_t(float b, R o, R inv, R oi)
{
    if constexpr (kFused) return fma(R(b), inv, -oi);
    else return (R(b) - o) * inv;
}

// Slab tests of the four child boxes against [tlo, thi]; tn is the entry
// distance clamped to tlo.  The boxes are padded at build time, so rounding
// never loses a hit.  The node words come in the ray's octant order, and the
// rounded plane distance is monotonic in the plane coordinate, so each
// near-plane distance is exactly the smaller of the axis's two (and the far
// one the larger): the same values a min/max of the pair gives.
// Empty child slots hold inverted boxes (lower planes +inf, upper -inf), whose
// entry distance is +inf and exit -inf for every ray, so no test of the
// child's entry is needed (a NaN ray that took one would find a leaf of no
// triangles).
template <bool kFused, class R>
__device__ __forceinline__ void box4(const WideNode &nd, const Ray<R> &ry, R tlo, R thi, R (&tn)[4],
                                     bool (&hit)[4])
{
    const V3<R> o = ry.o, inv = ry.inv, oi = ry.oi;
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        const R ax = slab_t<kFused>(f4get(nd.nx, c), o.x, inv.x, oi.x), bx = slab_t<kFused>(f4get(nd.fx, c), o.x, inv.x, oi.x);
        const R ay = slab_t<kFused>(f4get(nd.ny, c), o.y, inv.y, oi.y), by = slab_t<kFused>(f4get(nd.fy, c), o.y, inv.y, oi.y);
        const R az = slab_t<kFused>(f4get(nd.nz, c), o.z, inv.z, oi.z), bz = slab_t<kFused>(f4get(nd.fz, c), o.z, inv.z, oi.z);
        const R a = fmax(fmax(ax, ay), fmax(az, tlo));
        const R b = fmin(fmin(bx, by), fmin(bz, thi));
        tn[c] = a;
        hit[c] = a <= b;
    }
}

// Compare-exchange of (key, entry) pairs by key.
__device__ __forceinline__ void cswap(uint32_t &ka, int32_t &ea, uint32_t &kb, int32_t &eb)
{
    const bool sw = kb < ka;
    const uint32_t k = sw ? kb : ka;
    const int32_t e = sw ? eb : ea;
    kb = sw ? ka : kb;
    eb = sw ? ea : eb;
    ka = k;
    ea = e;
}

// Children hit by the ray, nearest first: keys hold the entry distance's
// bits with the child slot in the two low bits (distances are >= teps > 0, so
// their bits order like the values; misses sort last); a five-exchange
// sorting network orders the (key, entry) pairs.  Returns the hit count.
template <class R>
__device__ __forceinline__ int order_children(const WideNode &nd, const R (&tn)[4], const bool (&hit)[4],
                                              int32_t (&e)[4])
{
    uint32_t k[4];
    int nh = 0;
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        k[c] = hit[c] ? ((__float_as_uint((float)tn[c]) & ~3u) | (uint32_t)c) : 0xFFFFFFFFu;
        e[c] = child_at(nd, c);
        nh += hit[c] ? 1 : 0;
    }
    cswap(k[0], e[0], k[1], e[1]);
    cswap(k[2], e[2], k[3], e[3]);
    cswap(k[0], e[0], k[2], e[2]);
    cswap(k[1], e[1], k[3], e[3]);
    cswap(k[1], e[1], k[2], e[2]);
    return nh;
}

template <class R>
struct Closest {
    R tb, ub, vb;
    int32_t trib, orig_b;
};

template <class R>
__device__ __forceinline__ R teps_of(const SceneDev &sc)
{
    return sizeof(R) == 4 ? R(sc.teps_f) : R(sc.teps_d);
}

__device__ __forceinline__ TriDev load_tri(const TriDev *tris, int i)
{
    const float4 *p = reinterpret_cast<const float4 *>(tris) + 3 * (size_t)i;
    TriDev t;
    t.a = gld4(p);
    t.b = gld4(p + 1);
    t.c = gld4(p + 2);
    return t;
}

// One step of a closest-hit search: visit nodes, entering the nearest child
// box hit and stacking the others farthest first, until a leaf is due; test
// that leaf and report whether the search is complete.  Ties in t go to the
// smaller caller triangle index, so the result does not depend on the tree.
//
// Descent is speculative: a lane that reaches a leaf keeps it for the test
// and goes on with its stack while other lanes of the wave are still
// searching for theirs, so lanes do not idle through the longest descent of
// the wave (its extra visits use the larger bound of before the test, which
// changes no result); it may pick up a second leaf on the way, tested in the
// same step.  The descent ends when fewer than kDescentLanes lanes are still
// looking for a first leaf (after at least one round of visits); those lanes
// go on from where they stopped in the next step.
// kSkipCaller: ry.skip holds the caller index of the triangle to skip (the
// tree's triangles are copies, as in a sub-domain's cell), not its position.
template <bool kFused, class R, class St, bool kSkipCaller = false>
__device__ __forceinline__ bool closest_step(const SceneDev &sc, const float4 *lds_nodes, int n_lds, St &st,
                                             Ray<R> &ry, Closest<R> &h, R teps, uint32_t &nodes, uint32_t &tests)
{
    int32_t cur = ry.cur;      // inner node (>= 0), leaf (< -1) or kDone
    int32_t leaf = kDone, leaf2 = kDone;
    bool visited = false;
    for (;;) {
        if (cur < 0 && cur != kDone && leaf2 == kDone) {
            if (leaf == kDone) leaf = cur;
            else leaf2 = cur;
            cur = st.sp ? st.pop() : kDone;
        }
        const uint64_t searching = wave_ballot(leaf == kDone && cur >= 0);
        if (!searching) break;
        // after one round of visits (so every step advances every lane), the
        // few lanes still searching resume in the next step rather than hold
        // the wave's leaf tests back
        if (visited && __popcll(searching) < kDescentLanes) break;
        visited = true;
        if (cur >= 0) {
            const WideNode nd = load_node(lds_nodes, n_lds, sc.nodes, cur, ry.kx, ry.ky, ry.kz);
            ++nodes;
            R tn[4];
            bool hit[4];
            box4<kFused>(nd, ry, teps, h.tb, tn, hit);
            int32_t e[4];
            const int nh = order_children(nd, tn, hit, e);
            if (nh == 0) {
                cur = st.sp ? st.pop() : kDone;
            } else {
                st.push_sorted(nh - 1, e[1], e[2], e[3]);
                cur = e[0];
            }
        }
    }
    {
        // the triangles of both leaves held, in one loop
        const int32_t ca = leaf != kDone ? -1 - leaf : 0, cb = leaf2 != kDone ? -1 - leaf2 : 0;
        const int fa = ca >> 8, na = ca & 255, fb = cb >> 8, nb = cb & 255;
        tests += (uint32_t)(na + nb);
        // a sub-domain cell's walk reads its cell's copies in scene coordinates:
        // rotated copies of every cell's triangles would triple a footprint
        // that is already spread over many cells, which costs more in cache
        // misses than the per-lane coordinate selection saves
        const TriDev *tt = kSkipCaller ? sc.tris : test_tris(sc, ry);
        for (int k = 0; k < na + nb; ++k) {
            const int i = k < na ? fa + k : fb + (k - na);
            if (!kSkipCaller && i == ry.skip) continue;
            const TriDev tr = load_tri(tt, i);
            const int32_t orig = __float_as_int(tr.a.w);
            if (kSkipCaller && orig == ry.skip) continue;
            R t, u, v;
            if (!(kSkipCaller ? ray_tri(ry, from4<R>(tr.a), from4<R>(tr.b), from4<R>(tr.c), t, u, v)
                              : ray_tri_frame(ry, from4<R>(tr.a), from4<R>(tr.b), from4<R>(tr.c), t, u, v)))
                continue;
            if (!(t > teps)) continue;
            if (t < h.tb || (t == h.tb && orig < h.orig_b)) {
                h.tb = t; h.trib = i; h.ub = u; h.vb = v; h.orig_b = orig;
            }
        }
    }
    ry.cur = cur;
    return cur == kDone;
}

// One step of an any-hit walk toward +infinity: visit nodes until a leaf is
// due (speculatively, as in the closest-hit step) and test it.  An opaque
// triangle ends the walk (occluded); each pane crossed is reported to
// on_glass(leaf, material, u, v).
template <bool kFused, class R, class St, class F>
__device__ __forceinline__ bool shadow_step(const SceneDev &sc, const float4 *lds_nodes, int n_lds, St &st,
                                            Ray<R> &ry, bool &occluded, R teps, F &&on_glass, uint32_t &nodes,
                                            uint32_t &tests)
{
    const R tinf = R(INFINITY);
    int32_t cur = ry.cur;
    int32_t leaf = kDone;
    for (;;) {
        if (cur < 0 && cur != kDone && leaf == kDone) {
            leaf = cur;
            cur = st.sp ? st.pop() : kDone;
        }
        if (!wave_ballot(leaf == kDone && cur >= 0)) break;
        if (cur >= 0) {
            const WideNode nd = load_node(lds_nodes, n_lds, sc.nodes, cur, ry.kx, ry.ky, ry.kz);
            ++nodes;
            R tn[4];
            bool hit[4];
            box4<kFused>(nd, ry, teps, tinf, tn, hit);
            // any order finds every pane: enter the first child hit, stack the others
            int32_t nxt = kDone;
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                if (!hit[c]) continue;
                const int32_t e = child_at(nd, c);
                if (nxt == kDone) nxt = e;
                else st.push(e);
            }
            cur = nxt != kDone ? nxt : (st.sp ? st.pop() : kDone);
        }
    }
    if (leaf != kDone) {
        const int32_t code = -1 - leaf;
        const int first = code >> 8, cnt = code & 255;
        tests += (uint32_t)cnt;
        const TriDev *tt = test_tris(sc, ry);
        for (int i = first; i < first + cnt; ++i) {
            if (i == ry.skip) continue;
            const TriDev tr = load_tri(tt, i);
            R t, u, v;
            if (!ray_tri_frame(ry, from4<R>(tr.a), from4<R>(tr.b), from4<R>(tr.c), t, u, v)) continue;
            if (!(t > teps)) continue;
            const int mt = __float_as_int(tr.c.w);
            if (mt == 0 || mt == 3) {   // Lambert (spectral or gray): opaque
                occluded = true;
                ry.cur = kDone;
                return true;
            }
            on_glass(i, __float_as_int(tr.b.w), u, v);
        }
    }
    ry.cur = cur;
    return cur == kDone;
}

// Sun-grid walk of a shadow ray (scenes with a sun grid): the candidates of
// the ray's cell, by increasing smallest depth, up to kGridBatch per step.
// Candidates entirely behind the origin are skipped; the triangle test
// decides the rest exactly as in the BVH walk, and the first opaque triangle
// crossed ends the walk.
constexpr uint32_t kGridBatch = 8;

template <class R>
struct GridRange {
    uint32_t cur, end;
    R depth;             // o . sun, less the padding
};

template <class R>
__device__ __forceinline__ GridRange<R> grid_range(const SceneDev &sc, V3<R> o)
{
    GridRange<R> g;
    const R a = o.x * R(sc.g_e1[0]) + o.y * R(sc.g_e1[1]) + o.z * R(sc.g_e1[2]);
    const R b = o.x * R(sc.g_e2[0]) + o.y * R(sc.g_e2[1]) + o.z * R(sc.g_e2[2]);
    g.depth = o.x * R(sc.sun[0]) + o.y * R(sc.sun[1]) + o.z * R(sc.sun[2]) - R(sc.g_marg);
    const R fx = (a - R(sc.g_u0)) * R(sc.g_idu), fy = (b - R(sc.g_v0)) * R(sc.g_idv);
    g.cur = g.end = 0;
    // outside the grid no padded projection covers the point
    if (fx >= R(0) && fx < R(sc.g_nx) && fy >= R(0) && fy < R(sc.g_ny)) {
        const int c = (int)fx + sc.g_nx * (int)fy;
        g.cur = (uint32_t)gld(sc.g_start + c);
        g.end = (uint32_t)gld(sc.g_start + c + 1);
    }
    return g;
}

template <class R, class F>
__device__ __forceinline__ bool grid_step(const SceneDev &sc, const Ray<R> &ry, GridRange<R> &g, bool &occluded,
                                          R teps, F &&on_glass, uint32_t &cands, uint32_t &tests)
{
    const uint32_t stop = min(g.end, g.cur + kGridBatch);
    // FP32 reads the candidates rotated into the frame of the sun's dominant
    // axis, the frame of every shadow ray's test (the scene's other rays
    // never walk the grid)
    bool framed = false;
    if constexpr (sizeof(R) == 4) framed = ry.sh.kz == (uint32_t)sc.g_rot;
    const GridCand *cand = framed ? sc.g_cand_rot : sc.g_cand;
    for (; g.cur < stop; ++g.cur) {
        const float4 *cp = reinterpret_cast<const float4 *>(cand) + 3 * (size_t)g.cur;
        const float4 A = gld4(cp), B = gld4(cp + 1), C = gld4(cp + 2);
        ++cands;
        const int leaf = __float_as_int(A.w);
        if (R(B.w) < g.depth || leaf == ry.skip) continue;
        ++tests;
        R t, u, v;
        if (!(framed ? ray_tri_frame(ry, from4<R>(A), from4<R>(B), from4<R>(C), t, u, v)
                     : ray_tri(ry, from4<R>(A), from4<R>(B), from4<R>(C), t, u, v)))
            continue;
        if (!(t > teps)) continue;
        const int mw = __float_as_int(C.w), mt = mw & 3;
        if (mt == 0 || mt == 3) {   // Lambert (spectral or gray): opaque
            occluded = true;
            g.cur = g.end;
            return true;
        }
        on_glass(leaf, mw >> 2, u, v);
    }
    return g.cur >= g.end;
}

// Work distribution of the persistent traversal kernels: wave w of W takes
// the kFetch-item groups w, w + W, w + 2W, ... and hands their items to its
// idle lanes as they finish.  The interleaving spreads costly regions of the
// ray buffer over all waves; a shared claim counter, hit by every wave of all
// XCDs, costs more than the balance it buys.
struct WaveFeed {
    uint32_t beg, end;
    bool done;
    uint32_t group;      // groups taken so far
    // All lanes call this together; returns the item of an idle lane or -1.
    __device__ __forceinline__ int64_t next(bool idle, uint32_t count)
    {
        const uint64_t m = __ballot(idle);
        if (!m || done) return -1;
        if (beg >= end) {
            const uint32_t nw = (gridDim.x * blockDim.x) >> 6;
            const uint32_t wid = (blockIdx.x * blockDim.x + threadIdx.x) >> 6;
            const uint64_t base = ((uint64_t)wid + (uint64_t)group * nw) * kFetch;
            ++group;
            if (base >= count) {
                done = true;
                return -1;
            }
            beg = (uint32_t)base;
            end = (uint32_t)min<uint64_t>(base + kFetch, count);
        }
        const uint32_t before = (uint32_t)__popcll(m & ((1ull << lane_id()) - 1ull));
        const int64_t item = (idle && beg + before < end) ? (int64_t)(beg + before) : -1;
        beg = min(end, beg + (uint32_t)__popcll(m));
        return item;
    }
};

template <class R>
__device__ __forceinline__ V3<R> tri_normal(const TriDev &tr)
{
    const V3<R> p0 = from4<R>(tr.a), p1 = from4<R>(tr.b), p2 = from4<R>(tr.c);
    return normalize(cross(p1 - p0, p2 - p0));
}

template <class R>
__device__ __forceinline__ R pane_thickness(const SceneDev &sc, int leaf, int mat, R u, R v)
{
    if (!sc.has_vthick) return R(gld(sc.mat_thick + mat));
    const float4 th = gld4(sc.thick + leaf);
    return (R(1) - u - v) * R(th.x) + u * R(th.y) + v * R(th.z);
}

// Material and thickness of a pane at barycentric (u, v) of leaf-order
// triangle `leaf` whose own material is `mat`: with a distribution map (Sec.
// 6), the material of the texel under the hit's texture coordinates and, if
// the map has one, the bilinear thickness of its texel centres (clamped at
// the edges); otherwise `mat` and the triangle's thickness.
template <class R>
__device__ __forceinline__ void pane_at(const SceneDev &sc, int leaf, int mat, R u, R v, int &m_out, R &d_out)
{
    m_out = mat;
    const int mp = sc.n_maps > 0 ? gld(sc.mat_map + mat) : -1;
    if (mp < 0) {
        d_out = pane_thickness<R>(sc, leaf, mat, u, v);
        return;
    }
    const int4 hdr = gld4(sc.map_hdr + mp);
    const float4 q01 = gld4(sc.tri_uv + 2 * leaf), q2 = gld4(sc.tri_uv + 2 * leaf + 1);
    const R w0 = R(1) - u - v;
    const R s = w0 * R(q01.x) + u * R(q01.z) + v * R(q2.x);
    const R t = w0 * R(q01.y) + u * R(q01.w) + v * R(q2.y);
    const int W = hdr.x, H = hdr.y;
    const R fs = floor(s * R(W)), ft = floor(t * R(H));
    const int ix = fs < R(0) ? 0 : (fs > R(W - 1) ? W - 1 : (int)fs);
    const int iy = ft < R(0) ? 0 : (ft > R(H - 1) ? H - 1 : (int)ft);
    m_out = gld(sc.map_mat + hdr.z + iy * W + ix);
    if (!hdr.w) {
        d_out = pane_thickness<R>(sc, leaf, mat, u, v);
        return;
    }
    const R xs = s * R(W) - R(0.5), ys = t * R(H) - R(0.5);
    const R x0 = floor(xs), y0 = floor(ys), fx = xs - x0, fy = ys - y0;
    auto cl = [](R a, int n) { return a < R(0) ? 0 : (a > R(n - 1) ? n - 1 : (int)a); };
    const int xa = cl(x0, W), xb = cl(x0 + R(1), W), ya = cl(y0, H), yb = cl(y0 + R(1), H);
    const float *T = sc.map_thick + hdr.z;
    const R t00 = R(gld(T + ya * W + xa)), t10 = R(gld(T + ya * W + xb));
    const R t01 = R(gld(T + yb * W + xa)), t11 = R(gld(T + yb * W + xb));
    d_out = (R(1) - fy) * ((R(1) - fx) * t00 + fx * t10) + fy * ((R(1) - fx) * t01 + fx * t11);
}

// ---------------------------------------------------------------------------
// Camera rays (Sec. 3.1: a ray from each pixel).  Image point ((i + u0) / W,
// (j + u1) / H), row j from the top; pinhole through the unit-distance image
// plane, or orthographic rays along the view axis.
// ---------------------------------------------------------------------------
template <class R>
__global__ void __launch_bounds__(kBlock) k_generate(const JobDev *__restrict__ jobs, const BandDev *__restrict__ bands,
                                                     const ItemDev *items, int32_t n_items, Work<R> w,
                                                     uint64_t total, uint32_t chunk)
{
    // the chunk starts at the device cursor, so every chunk launches the same
    // kernel sequence with the same arguments (a graph replays it)
    const uint64_t r0 = w.cnt->r0;
    const uint32_t n = (uint32_t)min((uint64_t)chunk, total - min(r0, total));
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        if (n > 0) {
            int lo = 0, hi = n_items - 1;
            while (lo < hi) {
                const int mid = (lo + hi + 1) >> 1;
                if (items[mid].first <= r0) lo = mid; else hi = mid - 1;
            }
            w.cnt->lds_job = bands[items[lo].band].job;
        }
        w.cnt->count[0] = n;
        w.cnt->ddn[1] = 0;      // the first sub-domain pass's output queue
        w.cnt->count[1] = 0;
        w.cnt->scount = w.cnt->kcount = w.cnt->gcount = w.cnt->bcount = 0;
    }
    const Pool<R> P = w.p[0];
    const uint32_t stride = gridDim.x * blockDim.x;
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        const uint64_t r = r0 + i;
        int lo = 0, hi = n_items - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (items[mid].first <= r) lo = mid; else hi = mid - 1;
        }
        const ItemDev it = items[lo];
        const uint32_t l = (uint32_t)(r - it.first);
        const uint32_t pip = l / (uint32_t)it.ns;
        const uint32_t smp = (uint32_t)it.s0 + l % (uint32_t)it.ns;
        const int px = it.x0 + (int)(pip % (uint32_t)it.tw), py = it.y0 + (int)(pip / (uint32_t)it.tw);
        const BandDev bd = bands[it.band];
        const JobDev &jb = jobs[bd.job];
        const uint32_t pixel = (uint32_t)(py * jb.W + px);
        const uint4 rr = vertex_draws(jb.seed, jb.job_word, pixel, smp, -1, 0);
        const R x = (R(px) + u01<R>(rr.x)) / R(jb.W), y = (R(py) + u01<R>(rr.y)) / R(jb.H);
        const R a = R(2) * x - R(1), b = R(1) - R(2) * y;
        V3<R> o, d;
        const V3<R> f = {R(jb.f[0]), R(jb.f[1]), R(jb.f[2])};
        const V3<R> rv = {R(jb.r[0]), R(jb.r[1]), R(jb.r[2])};
        const V3<R> uv = {R(jb.u[0]), R(jb.u[1]), R(jb.u[2])};
        const V3<R> eye = {R(jb.eye[0]), R(jb.eye[1]), R(jb.eye[2])};
        if (jb.projection == 1) {
            o = eye + (a * R(jb.oh) * R(jb.aspect)) * rv + (b * R(jb.oh)) * uv;
            d = f;
        } else {
            o = eye;
            d = normalize(f + (a * R(jb.th) * R(jb.aspect)) * rv + (b * R(jb.th)) * uv);
        }
        // all wavelengths start with weight 1: no kSpectral
        put_path<R>(P, i, o, d, -1, pixel, smp, pack_aux(0, it.band, bd.job), R(1));
    }
}

// ---------------------------------------------------------------------------
// Closest hit of every path of pool `cur`.
// ---------------------------------------------------------------------------
// kSurface: every ray of the pool starts inside the scene's bounds (after
// the first bounce, or camera rays of pinhole eyes within the bounds of the
// scene's triangles), so the fused slab form applies; other camera rays take
// the plain form.  kOne: the
// launch renders one job, so the scene's constants are uniform (scalar loads
// hoisted out of the loops) rather than looked up per lane.
template <class R, bool kSurface, bool kOne>
__global__ void __launch_bounds__(kTraceBlock) k_trace(const JobDev *__restrict__ jobs, Work<R> w, int cur, int lds_job)
{
    if (lds_job < -1) lds_job = w.cnt->lds_job;   // the job of the chunk's first path
    __shared__ float4 s_nodes[8 * kTraceNodes];
    __shared__ int32_t s_stack[kLdsStack * kTraceBlock];
    const uint32_t count = min(w.cnt->count[cur], w.cap);   // the counter may pass cap on overflow
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        w.cnt->count[cur ^ 1] = 0;
        w.cnt->closest += count;
    }
    const int n_lds = lds_job >= 0 ? stage_nodes(s_nodes, jobs[lds_job].sc, kTraceNodes) : 0;
    StackT<kTraceBlock> st = make_stack<kTraceBlock>(s_stack, w.gstack);
    const Pool<R> P = w.p[cur];
    WaveFeed feed{0, 0, false, 0};
    Ray<R> ry;
    Closest<R> h;
    int64_t item = -1;
    int job = 0;
    R teps = R(0);
    uint32_t n_nodes = 0, n_tests = 0;
    for (;;) {
        const int64_t got = feed.next(item < 0, count);
        if (got >= 0) {
            item = got;
            const uint32_t s = (uint32_t)got;
            job = kOne ? 0 : (int)(rec_load(P.s + s).aux >> kAuxJobShift);
            const SceneDev &sc = jobs[job].sc;
            const PathO<R> po = rec_load(P.o + s);
            const PathD<R> pd = rec_load(P.d + s);
            set_dir(ry, V3<R>{po.x, po.y, po.z}, V3<R>{pd.x, pd.y, pd.z});
            ry.skip = po.skip;
            ry.cur = sc.n_nodes > 0 ? 0 : kDone;
            teps = teps_of<R>(sc);
            h.tb = R(INFINITY); h.ub = h.vb = R(0); h.trib = -1; h.orig_b = INT_MAX;
            st.sp = 0;
        }
        if (!__ballot(item >= 0)) {
            if (feed.done) break;
            continue;
        }
        if (item >= 0) {
            const bool fin = ry.cur == kDone ||
                             closest_step<kSurface>(jobs[job].sc, s_nodes, job == lds_job ? n_lds : 0, st, ry, h, teps, n_nodes,
                                          n_tests);
            if (fin) {
                HitRec<R> hr;
                hr.t = h.tb; hr.u = h.ub; hr.v = h.vb; hr.tri = h.trib;
                rec_store(w.hit + item, hr);
                item = -1;
            }
        }
    }
    if (n_nodes) {
        atomicAdd(&w.cnt->nodes[0], (unsigned long long)n_nodes);
        atomicAdd(&w.cnt->tris[0], (unsigned long long)n_tests);
    }
}

// ---------------------------------------------------------------------------
// Closest hit by geometric sub-domains (Sec. 5).  The scene's bounds are cut
// into a grid of cells, each with its own BVH over the triangles that overlap
// it.  A ray is traced in one cell at a time, over its segment inside the
// cell: a hit before the ray's exit from the cell is the closest hit, since
// every nearer point of the ray lies in cells already searched.  A ray that
// leaves the cell without a hit crosses the interface to the next cell
// along its direction, carrying its state (pool slot, entry parameter;
// origin and direction stay in the pool).  Each pass takes the rays queued
// at the interfaces; the first takes every path of the pool and finds its
// cell.  Pass k reads queue counter ddn[k mod 3], appends to ddn[(k + 1)
// mod 3] and clears ddn[(k + 2) mod 3] for the pass after next; the passes
// per bounce are a multiple of 3, so the last one leaves ddn[1] clear for
// the next bounce's first pass (k_generate clears it before a chunk).
// ---------------------------------------------------------------------------
// Parameter range [t0, t1] of the ray inside the box, and the axis through
// whose face it leaves.
template <class R>
__device__ __forceinline__ bool dd_box(const float lo[3], const float hi[3], const Ray<R> &ry, R &t0, R &t1,
                                       int &axis)
{
    const R o[3] = {ry.o.x, ry.o.y, ry.o.z}, iv[3] = {ry.inv.x, ry.inv.y, ry.inv.z};
    t0 = R(0);
    t1 = R(INFINITY);
    axis = 0;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const R ta = (R(lo[a]) - o[a]) * iv[a], tb = (R(hi[a]) - o[a]) * iv[a];
        const R n = fmin(ta, tb), f = fmax(ta, tb);
        t0 = fmax(t0, n);
        if (f < t1) {
            t1 = f;
            axis = a;
        }
    }
    return t0 <= t1;
}

// kMarch: a ray that leaves a cell goes on in the neighbouring cell in the
// same thread (the hand-off stays in registers; one pass per bounce).
template <class R, bool kSurface, bool kFirst, bool kMarch>
__global__ void __launch_bounds__(kTraceBlock) k_dd_sweep(const JobDev *__restrict__ jobs, Work<R> w, int cur,
                                                          int pass, int last)
{
    __shared__ int32_t s_stack[kLdsStack * kTraceBlock];
    const SceneDev &sc = jobs[0].sc;
    const DdDev &dd = sc.dd;
    const Pool<R> P = w.p[cur];
    uint32_t n_in;
    if (kFirst) {
        n_in = min(w.cnt->count[cur], w.cap);
        if (blockIdx.x == 0 && threadIdx.x == 0) {
            w.cnt->count[cur ^ 1] = 0;
            w.cnt->closest += n_in;
            w.cnt->ddn[2] = 0;
        }
    } else {
        n_in = min(w.cnt->ddn[pass % 3], w.cap);
        if (blockIdx.x == 0 && threadIdx.x == 0) w.cnt->ddn[(pass + 2) % 3] = 0;
    }
    const DdEntry<R> *qin = w.ddq[(pass + 1) & 1];
    DdEntry<R> *qout = w.ddq[pass & 1];
    uint32_t *nout = &w.cnt->ddn[(pass + 1) % 3];
    StackT<kTraceBlock> st = make_stack<kTraceBlock>(s_stack, w.gstack);
    WaveFeed feed{0, 0, false, 0};
    Ray<R> ry;
    Closest<R> h;
    SceneDev cv = sc;            // the current cell's tree in the scene's place
    int64_t item = -1;
    uint32_t slot = 0;
    int32_t cell = -1;
    int axis = 0;
    const R teps = teps_of<R>(sc);
    uint32_t n_nodes = 0, n_tests = 0, n_cross = 0;
    for (;;) {
        const int64_t got = feed.next(item < 0, n_in);
        if (got >= 0) {
            item = got;
            if (kFirst) {
                slot = (uint32_t)got;
            } else {
                const DdEntry<R> e = qin[got];
                slot = e.slot;
                cell = e.cell;
            }
            const PathO<R> po = rec_load(P.o + slot);
            const PathD<R> pd = rec_load(P.d + slot);
            set_dir(ry, V3<R>{po.x, po.y, po.z}, V3<R>{pd.x, pd.y, pd.z});
            ry.skip = po.skip >= 0 ? __float_as_int(load_tri(sc.tris, po.skip).a.w) : -1;
            if (kFirst) {
                // the cell of the origin, or of the point where the ray
                // enters the grid
                const float glo[3] = {dd.lo[0], dd.lo[1], dd.lo[2]};
                const float ghi[3] = {dd.lo[0] + dd.size[0] * dd.n[0], dd.lo[1] + dd.size[1] * dd.n[1],
                                      dd.lo[2] + dd.size[2] * dd.n[2]};
                R g0, g1;
                int ax;
                cell = -1;
                if (dd_box(glo, ghi, ry, g0, g1, ax)) {
                    const R p[3] = {ry.o.x + g0 * ry.d.x, ry.o.y + g0 * ry.d.y, ry.o.z + g0 * ry.d.z};
                    int k[3];
#pragma unroll
                    for (int a = 0; a < 3; ++a) {
                        const R f = floor((p[a] - R(dd.lo[a])) / R(dd.size[a]));
                        k[a] = f < R(0) ? 0 : (f > R(dd.n[a] - 1) ? dd.n[a] - 1 : (int)f);
                    }
                    cell = (k[2] * dd.n[1] + k[1]) * dd.n[0] + k[0];
                }
            }
            h.tb = R(INFINITY); h.ub = h.vb = R(0); h.trib = -1; h.orig_b = INT_MAX;
            st.sp = 0;
            ry.cur = kDone;
            if (cell >= 0) {
                const CellDev c = dd.cells[cell];
                R t0, t1;
                dd_box(c.lo, c.hi, ry, t0, t1, axis);
                h.tb = t1;     // only hits before the ray leaves the cell
                cv.nodes = dd.nodes + c.node_base;
                cv.tris = dd.tris + c.tri_base;
                cv.n_nodes = c.n_nodes;
                ry.cur = c.n_nodes > 0 ? 0 : kDone;
            }
        }
        if (!__ballot(item >= 0)) {
            if (feed.done) break;
            continue;
        }
        if (item >= 0) {
            const bool fin = ry.cur == kDone ||
                             closest_step<kSurface, R, StackT<kTraceBlock>, true>(cv, nullptr, 0, st, ry, h, teps,
                                                                                 n_nodes, n_tests);
            if (fin) {
                HitRec<R> hr;
                hr.t = R(INFINITY); hr.u = hr.v = R(0); hr.tri = -1;
                int next = -1;
                if (h.trib >= 0) {
                    hr.t = h.tb; hr.u = h.ub; hr.v = h.vb;
                    hr.tri = gld(dd.leaf + dd.cells[cell].tri_base + h.trib);
                } else if (cell >= 0) {
                    // across the face of the exit axis, toward the ray's direction
                    int k[3] = {cell % dd.n[0], (cell / dd.n[0]) % dd.n[1], cell / (dd.n[0] * dd.n[1])};
                    const R da = axis == 0 ? ry.d.x : (axis == 1 ? ry.d.y : ry.d.z);
                    k[axis] += da > R(0) ? 1 : -1;
                    if (k[axis] >= 0 && k[axis] < dd.n[axis]) next = (k[2] * dd.n[1] + k[1]) * dd.n[0] + k[0];
                }
                if (kMarch && next >= 0) {
                    // continue in the neighbour from the interface
                    cell = next;
                    const CellDev c = dd.cells[cell];
                    R t0, t1;
                    dd_box(c.lo, c.hi, ry, t0, t1, axis);
                    h.tb = t1;
                    h.ub = h.vb = R(0); h.trib = -1; h.orig_b = INT_MAX;
                    cv.nodes = dd.nodes + c.node_base;
                    cv.tris = dd.tris + c.tri_base;
                    cv.n_nodes = c.n_nodes;
                    st.sp = 0;
                    ry.cur = c.n_nodes > 0 ? 0 : kDone;
                    ++n_cross;
                    continue;
                }
                if (next >= 0 && last) {
                    atomicOr(&w.cnt->overflow, 4u);   // more cells than the passes cover
                    next = -1;
                }
                if (next >= 0) {
                    const uint32_t q = atomicAdd(nout, 1u);
                    if (q < w.cap) {
                        DdEntry<R> e;
                        e.t = h.tb;
                        e.slot = slot;
                        e.cell = next;
                        qout[q] = e;
                    } else {
                        atomicOr(&w.cnt->overflow, 1u);
                    }
                    ++n_cross;
                } else {
                    rec_store(w.hit + slot, hr);
                }
                item = -1;
            }
        }
    }
    if (n_nodes) {
        atomicAdd(&w.cnt->nodes[0], (unsigned long long)n_nodes);
        atomicAdd(&w.cnt->tris[0], (unsigned long long)n_tests);
    }
    if (n_cross) atomicAdd(&w.cnt->interface_rays, (unsigned long long)n_cross);
}

// ---------------------------------------------------------------------------
// Caustic photon map (photon mapping, Sec. 3.2: a pass before the render
// shoots photons from the light and stores where they land; the render
// estimates the light they carry from their density).  Sun photons, each of
// one render wavelength, leave a square across the sun's direction that
// covers the scene and follow the panes' optics: clear glass reflects with
// probability R / (R + T) (weight R + T), bubbly glass takes the exact walk.
// A photon is stored where it first meets a Lambert surface if a pane has
// turned it (a reflection, or light scattered by bubbles): the straight,
// unscattered sunlight is the render's own shadow-ray estimate.  The stored
// photons are hashed by the cell of side r they lie in.
// ---------------------------------------------------------------------------

__device__ __forceinline__ uint32_t ph_hash(int ix, int iy, int iz, uint32_t mask)
{
    return (((uint32_t)ix * 73856093u) ^ ((uint32_t)iy * 19349663u) ^ ((uint32_t)iz * 83492791u)) & mask;
}

// Coarse cell (side 3 r) of a cell index: floor(i / 3), also below zero.
__device__ __forceinline__ int ph_coarse(int i) { return i >= 0 ? i / 3 : -((2 - i) / 3); }

template <class R>
__device__ __forceinline__ void ph_cell(const V3<R> &x, const double lo[3], double r, int &ix, int &iy, int &iz)
{
    const R ir = R(1.0 / r);
    ix = (int)floor((x.x - R(lo[0])) * ir);
    iy = (int)floor((x.y - R(lo[1])) * ir);
    iz = (int)floor((x.z - R(lo[2])) * ir);
}

template <class R>
__global__ void __launch_bounds__(kTraceBlock) k_photon(const JobDev *__restrict__ jobs, PhotonWork<R> pw)
{
    __shared__ int32_t s_stack[kLdsStack * kTraceBlock];
    const JobDev &jb = jobs[0];
    const SceneDev &sc = jb.sc;
    StackT<kTraceBlock> st = make_stack<kTraceBlock>(s_stack, pw.gstack);
    WaveFeed feed{0, 0, false, 0};
    Ray<R> ry;
    Closest<R> h;
    int64_t item = -1;
    uint32_t pid = 0;
    int vtx = 0, j = 0;
    bool turned = false;
    R phi = R(0);
    const R teps = teps_of<R>(sc);
    const V3<R> sun = {R(sc.sun[0]), R(sc.sun[1]), R(sc.sun[2])};
    uint32_t n_nodes = 0, n_tests = 0;
    for (;;) {
        const int64_t got = feed.next(item < 0, pw.n);
        if (got >= 0) {
            item = got;
            pid = (uint32_t)got;
            const uint4 e = vertex_draws(jb.seed, jb.job_word, pid, kPhotonTag, -1, 0);
            const R a = R(2) * u01<R>(e.x) - R(1), b = R(2) * u01<R>(e.y) - R(1);
            j = min((int)(u01<R>(e.z) * R(jb.nl)), jb.nl - 1);
            const V3<R> o = {R(pw.c[0]) + a * R(pw.e1[0]) + b * R(pw.e2[0]),
                             R(pw.c[1]) + a * R(pw.e1[1]) + b * R(pw.e2[1]),
                             R(pw.c[2]) + a * R(pw.e1[2]) + b * R(pw.e2[2])};
            set_dir(ry, o, R(-1) * sun);
            ry.skip = -1;
            phi = gld((const R *)jb.E + j) * R(pw.power);
            vtx = 0;
            turned = false;
            h.tb = R(INFINITY); h.ub = h.vb = R(0); h.trib = -1; h.orig_b = INT_MAX;
            st.sp = 0;
            ry.cur = sc.n_nodes > 0 ? 0 : kDone;
        }
        if (!__ballot(item >= 0)) {
            if (feed.done) break;
            continue;
        }
        if (item >= 0) {
            const bool fin = ry.cur == kDone || closest_step<false>(sc, nullptr, 0, st, ry, h, teps, n_nodes, n_tests);
            if (fin) {
                bool go = false;
                V3<R> x = ry.o, dn = ry.d;
                if (h.trib >= 0 && vtx < jb.max_depth && phi > R(0)) {
                    const TriDev tr = load_tri(sc.tris, h.trib);
                    const int mat = __float_as_int(tr.b.w), mt = __float_as_int(tr.c.w);
                    const V3<R> d = ry.d, ng = tri_normal<R>(tr);
                    x = ry.o + h.tb * d;
                    const R cos_i = fabs(dot(d, ng));
                    const R lam = gld((const R *)jb.lam + j);
                    if (mt == 0 || mt == 3) {
                        if (turned) {
                            const uint32_t q = atomicAdd(&pw.cnt->phcount, 1u);
                            if (q < pw.cap) {
                                const V3<R> ns = dot(ng, d) > R(0) ? R(-1) * ng : ng;
                                PhotonRec<R> pr;
                                pr.x = x.x; pr.y = x.y; pr.z = x.z; pr.phi = phi;
                                pr.nx = ns.x; pr.ny = ns.y; pr.nz = ns.z; pr.j = j;
                                pw.rec[q] = pr;
                            }
                        }
                    } else if (mt == 1) {
                        int me;
                        R thick;
                        pane_at<R>(sc, h.trib, mat, h.ub, h.vb, me, thick);
                        const size_t mo = (size_t)me * jb.ms + j;
                        R Rr, Tt;
                        slab_RT<R>(cos_i, lam, thick, gld((const R *)jb.n + mo), gld((const R *)jb.k + mo),
                                   gld((const R *)jb.tint + mo), Rr, Tt);
                        const R u = u01<R>(vertex_draws(jb.seed, jb.job_word, pid, kPhotonTag, vtx, 0).x);
                        if (Rr + Tt > R(0) && u < Rr / (Rr + Tt)) {
                            dn = d - (R(2) * dot(d, ng)) * ng;
                            turned = true;
                        }
                        phi *= Rr + Tt;
                        go = true;
                    } else {
                        // bubbly pane: the exact walk at the photon's wavelength
                        const R thick = pane_thickness<R>(sc, h.trib, mat, h.ub, h.vb);
                        const double *bub = sc.mat_bub + 4 * (size_t)mat;
                        const size_t mo = (size_t)mat * jb.ms + j;
                        const R nn = gld((const R *)jb.n + mo), kk = gld((const R *)jb.k + mo);
                        const WalkStream ws = {jb.seed, pid, kPhotonTag, jb.job_word, (uint32_t)vtx, true};
                        R ue[4];
                        walk_draw<R>(ws, 0, 0, ue);
                        const int pol = ue[1] < R(0.5) ? 0 : 1;
                        R Rs, Rp;
                        fresnel_sp<R>(cos_i, nn, kk, Rs, Rp);
                        if (ue[0] < (pol == 0 ? Rs : Rp)) {
                            dn = d - (R(2) * dot(d, ng)) * ng;
                            turned = true;
                            go = true;
                        } else {
                            const WalkOut<R> wo = bubbly_walk<R>(ws, cos_i, thick, R(gld(bub)), R(gld(bub + 1)), pol);
                            if (wo.kind != 0) {
                                dn = slab_to_world<R>(d, ng, wo.a);
                                turned = turned || wo.kind == 1 || wo.bubbles > 0;
                                const R alpha = R(12.566370614359172) * kk / (lam * R(1e-6)) +
                                                gld((const R *)jb.tint + mo);
                                phi *= exp(-alpha * wo.L);
                                go = true;
                            }
                        }
                    }
                    ++vtx;
                }
                if (go && vtx < jb.max_depth) {
                    set_dir(ry, x, dn);
                    ry.skip = h.trib;
                    h.tb = R(INFINITY); h.ub = h.vb = R(0); h.trib = -1; h.orig_b = INT_MAX;
                    st.sp = 0;
                    ry.cur = sc.n_nodes > 0 ? 0 : kDone;
                } else {
                    item = -1;
                }
            }
        }
    }
}

// Hash grid: clear the counts and cursors, count the photons per bucket,
// scan (blocks of 4096, then the block sums), and place each photon.
template <class R>
__global__ void __launch_bounds__(kBlock) k_ph_clear(PhotonWork<R> pw)
{
    const uint32_t n = max(pw.mask + 2u, kPhCoarseWords);
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        if (i <= pw.mask + 1u) pw.start[i] = 0u;
        if (i <= pw.mask) pw.cursor[i] = 0u;
        if (i <= pw.occ_mask >> 5) pw.occ[i] = 0u;
        if (i < kPhCoarseWords) pw.cocc[i] = 0u;
    }
}

template <class R>
__global__ void __launch_bounds__(kBlock) k_ph_count(PhotonWork<R> pw)
{
    const uint32_t n = min(pw.cnt->phcount, pw.cap);
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        const PhotonRec<R> p = pw.rec[i];
        int ix, iy, iz;
        ph_cell<R>(V3<R>{p.x, p.y, p.z}, pw.lo, pw.r, ix, iy, iz);
        const uint32_t b = ph_hash(ix, iy, iz, pw.mask);
        atomicAdd(pw.start + b, 1u);
        atomicOr(pw.occ + ((b & pw.occ_mask) >> 5), 1u << (b & 31u));
        const uint32_t cb = ph_hash(ph_coarse(ix), ph_coarse(iy), ph_coarse(iz), kPhCoarseBits - 1u);
        atomicOr(pw.cocc + (cb >> 5), 1u << (cb & 31u));
    }
}

constexpr int kScanBlock = 1024, kScanPer = 4;   // 4096 values per block

// Exclusive scan of v[0, n) in blocks of 4096; each block's total to part.
__global__ void __launch_bounds__(kScanBlock) k_scan_blocks(uint32_t *v, uint32_t n, uint32_t *part)
{
    __shared__ uint32_t s[kScanBlock];
    const uint32_t base = blockIdx.x * (kScanBlock * kScanPer) + threadIdx.x * kScanPer;
    uint32_t x[kScanPer], sum = 0;
    for (int k = 0; k < kScanPer; ++k) {
        x[k] = base + k < n ? v[base + k] : 0u;
        sum += x[k];
    }
    s[threadIdx.x] = sum;
    __syncthreads();
    for (int off = 1; off < kScanBlock; off <<= 1) {    // inclusive scan of the thread sums
        const uint32_t t = threadIdx.x >= (uint32_t)off ? s[threadIdx.x - off] : 0u;
        __syncthreads();
        s[threadIdx.x] += t;
        __syncthreads();
    }
    uint32_t run = s[threadIdx.x] - sum;
    for (int k = 0; k < kScanPer; ++k) {
        if (base + k < n) v[base + k] = run;
        run += x[k];
    }
    if (part && threadIdx.x == kScanBlock - 1) part[blockIdx.x] = s[kScanBlock - 1];
}

__global__ void __launch_bounds__(kScanBlock) k_scan_add(uint32_t *v, uint32_t n, const uint32_t *part)
{
    const uint32_t add = part[blockIdx.x];
    const uint32_t base = blockIdx.x * (kScanBlock * kScanPer) + threadIdx.x * kScanPer;
    for (int k = 0; k < kScanPer; ++k)
        if (base + k < n) v[base + k] += add;
}

template <class R>
__global__ void __launch_bounds__(kBlock) k_ph_place(PhotonWork<R> pw)
{
    const uint32_t n = min(pw.cnt->phcount, pw.cap);
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        const PhotonRec<R> p = pw.rec[i];
        int ix, iy, iz;
        ph_cell<R>(V3<R>{p.x, p.y, p.z}, pw.lo, pw.r, ix, iy, iz);
        const uint32_t b = ph_hash(ix, iy, iz, pw.mask);
        pw.sorted[pw.start[b] + atomicAdd(pw.cursor + b, 1u)] = p;
    }
}

// Caustic gather at the Lambert vertices of the chunk (their shadow records):
// L_j += g b_j rho_j / pi * sum of Phi / (pi r^2) over the photons of
// wavelength j within r that arrived on the same side (normals within 0.9).
template <class R>
__global__ void __launch_bounds__(kBlock) k_caustic(const JobDev *__restrict__ jobs, const BandDev *__restrict__ bands,
                                                    Work<R> w, PhotonWork<R> pw)
{
    __shared__ uint32_t s_cocc[kPhCoarseWords];
    for (uint32_t i = threadIdx.x; i < kPhCoarseWords; i += blockDim.x) s_cocc[i] = pw.cocc[i];
    __syncthreads();
    const uint32_t ns = min(w.cnt->scount, w.cap);
    const JobDev &jb = jobs[0];
    const R r2 = R(pw.r * pw.r), inv_area = R(1.0 / (3.14159265358979323846 * pw.r * pw.r));
    const PhotonRec<R> *P = pw.sorted;
    for (uint32_t rec = blockIdx.x * blockDim.x + threadIdx.x; rec < ns; rec += gridDim.x * blockDim.x) {
        const uint32_t sp = w.spix[rec], aux = w.saux[rec];
        const BandDev bd = bands[(aux >> kAuxBandShift) & ((1u << kAuxBandBits) - 1u)];
        const bool spec = (sp & kSpectral) != 0u;
        const R gr = w.sgr[rec];
        if (gr == R(0)) continue;
        const V3<R> x = {w.sx[rec], w.sy[rec], w.sz[rec]}, n = {w.snx[rec], w.sny[rec], w.snz[rec]};
        double *row = w.acc + jb.acc_off + (uint64_t)(sp & ~kSpectral) * jb.nl;
        int cx, cy, cz;
        ph_cell<R>(x, pw.lo, pw.r, cx, cy, cz);
        // the 27 cells lie in at most 2 x 2 x 2 coarse cells: none holding a
        // photon (the common case) ends the record with LDS lookups only
        bool any = false;
        for (int gz = ph_coarse(cz - 1); gz <= ph_coarse(cz + 1); ++gz)
            for (int gy = ph_coarse(cy - 1); gy <= ph_coarse(cy + 1); ++gy)
                for (int gx = ph_coarse(cx - 1); gx <= ph_coarse(cx + 1); ++gx) {
                    const uint32_t cb = ph_hash(gx, gy, gz, kPhCoarseBits - 1u);
                    any = any || ((s_cocc[cb >> 5] >> (cb & 31u)) & 1u);
                }
        if (!any) continue;
        // occupancy of the 27 cells around x: every bitmap load issued before
        // any is tested (most cells are empty: one L2 round trip, not 27)
        auto cell_bucket = [&](int q) {
            return ph_hash(cx + q % 3 - 1, cy + (q / 3) % 3 - 1, cz + q / 9 - 1, pw.mask);
        };
        uint32_t occ27 = 0;
#pragma unroll
        for (int q = 0; q < 27; ++q) {
            const uint32_t b = cell_bucket(q);
            occ27 |= ((pw.occ[(b & pw.occ_mask) >> 5] >> (b & 31u)) & 1u) << q;
        }
        // each bucket once (cells may share one): skip a cell whose bucket an
        // earlier occupied cell has
        for (uint32_t mq = occ27; mq; mq &= mq - 1u) {
            const int q = __builtin_ctz(mq);
            const uint32_t b = cell_bucket(q);
            bool dup = false;
            for (uint32_t me = occ27 & ((1u << q) - 1u); me; me &= me - 1u) dup = dup || cell_bucket(__builtin_ctz(me)) == b;
            if (dup) continue;
            for (uint32_t k = pw.start[b]; k < pw.start[b + 1]; ++k) {
                const PhotonRec<R> p = P[k];
                if (p.j < bd.l0 || p.j >= bd.l0 + bd.nb) continue;
                const R ex = p.x - x.x, ey = p.y - x.y, ez = p.z - x.z;
                if (!(ex * ex + ey * ey + ez * ez < r2)) continue;
                if (!(p.nx * n.x + p.ny * n.y + p.nz * n.z > R(0.9))) continue;
                const R f = spec ? w.contrib[aosoa(rec, p.j - bd.l0, w.nbmax)] : R(1);
                unsafeAtomicAdd(row + p.j, (double)(gr * f * p.phi * inv_area));
            }
        }
    }
}

// ---------------------------------------------------------------------------
// Per-wavelength rows handled by the whole wave.  Each lane whose flag is set
// owns a task on rows of nbm values (nbm a multiple of 4); the wave works
// through the tasks ng at a time, gl = nbm / 4 lanes per task and four
// wavelengths per lane, one 16-byte access each.  A row's cache lines are
// then read or written by one instruction, where a lane walking its own row
// 16 bytes per step leaves them partly written while other rows evict them.
// Called by every lane of the wave; s_map is the wave's 64-entry LDS table.
// ---------------------------------------------------------------------------
constexpr uint32_t kRowSrc = 1u, kRowRho = 2u, kRowRec = 4u, kRowKeep = 8u, kRowAl = 16u, kRowFork = 32u;
constexpr int kRowNbShift = 8;   // band size in bits 8..15 of a task's flags
struct RowTasks {
    int n;              // tasks in the wave
    int gl, ng;         // lanes per task, tasks per step
    int sub;            // this lane's task within a step (idle when >= ng)
    int j;              // first of this lane's four wavelengths
    uint32_t rank;      // this lane's own task number (lanes with a task)
    __device__ __forceinline__ bool busy(int base) const { return sub < ng && base + sub < n; }
    // the lane owning the task this lane works on at step `base` (itself when idle)
    __device__ __forceinline__ int src(int base, const uint32_t *s_map) const
    {
        return busy(base) ? (int)s_map[min(base + sub, 63)] : (int)lane_id();
    }
    // whether this lane's own task is in step `base`, and its lanes there
    __device__ __forceinline__ bool mine(bool want, int base, uint64_t &lanes) const
    {
        const uint32_t s = rank - (uint32_t)base;
        if (!want || s >= (uint32_t)ng) return false;
        lanes = (gl == 64 ? ~0ull : ((1ull << gl) - 1ull)) << (s * gl);
        return true;
    }
};

__device__ __forceinline__ RowTasks row_tasks(bool want, int nbm, uint32_t *s_map)
{
    const uint32_t lane = lane_id();
    const uint64_t m = __ballot(want);
    RowTasks t;
    t.rank = (uint32_t)__popcll(m & ((1ull << lane) - 1ull));
    if (want) s_map[t.rank] = lane;
    __builtin_amdgcn_wave_barrier();
    t.n = __popcll(m);
    t.gl = nbm >> 2;
    t.ng = 64 / t.gl;
    t.sub = (int)lane / t.gl;
    t.j = ((int)lane - t.sub * t.gl) * 4;
    return t;
}

// ---------------------------------------------------------------------------
// Shade: misses add the sky, Lambert vertices emit a shadow record (eq. (3))
// and bounce; survivors are compacted with their weights into the other
// pool.  Glass vertices are queued for k_shade_glass so that the costly
// per-wavelength slab optics run in dense waves.
// ---------------------------------------------------------------------------
// Block-wide reservation of output slots in Q queues: every thread of the
// block calls it (block-uniform control flow).  One atomic per queue and
// block instead of one per wave; slots keep lane order within the block.
// NW: waves per block.
template <int Q, int NW = kBlock / 64>
__device__ __forceinline__ void block_reserve(const bool (&want)[Q], uint32_t *const (&ctr)[Q], uint32_t (&slot)[Q],
                                              uint32_t *s_cnt, uint32_t *s_base)
{
    const uint32_t lane = lane_id(), wv = threadIdx.x >> 6;
    const uint64_t lt = (1ull << lane) - 1ull;
    uint32_t pre[Q];
#pragma unroll
    for (int q = 0; q < Q; ++q) {
        const uint64_t m = __ballot(want[q]);
        pre[q] = (uint32_t)__popcll(m & lt);
        if (lane == 0) s_cnt[wv * Q + q] = (uint32_t)__popcll(m);
    }
    __syncthreads();
    if (threadIdx.x < (unsigned)Q) {
        const int q = threadIdx.x;
        uint32_t total = 0;
        for (int w2 = 0; w2 < NW; ++w2) total += s_cnt[w2 * Q + q];
        s_base[q] = total ? atomicAdd(ctr[q], total) : 0u;
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < Q; ++q) {
        uint32_t off = s_base[q] + pre[q];
        for (uint32_t w2 = 0; w2 < wv; ++w2) off += s_cnt[w2 * Q + q];
        slot[q] = off;
    }
    __syncthreads();   // s_cnt and s_base are reused by the next call
}

// FP32: eight waves per SIMD (64 VGPRs) hide more of the pass's memory
// latency; the FP64 instantiation keeps its registers.  Blocks of 512
// threads: every block iteration reserves its output slots with one atomic
// per queue on counters shared by the whole chip, and those atomics (on the
// memory side) bounded the pass at 256 threads.
template <class R, bool kOne>
__global__ void __launch_bounds__(kShadeBlock) __attribute__((amdgpu_waves_per_eu(sizeof(R) == 4 ? 8 : 1))) k_shade(const JobDev *__restrict__ jobs, const BandDev *__restrict__ bands, Work<R> w, int cur)
{
    const uint32_t count = min(w.cnt->count[cur], w.cap);   // the counter may pass cap on overflow
    const Pool<R> Pi = w.p[cur], Po = w.p[cur ^ 1];
    const int nbm = w.nbmax;
    const uint32_t lane = lane_id();
    const R inv_pi = R(0.31830988618379067);
    __shared__ uint32_t s_cnt[(kShadeBlock / 64) * 5], s_base[5];
    __shared__ uint32_t s_map_all[kShadeBlock];
    uint32_t *const s_map = s_map_all + (threadIdx.x & ~63u);
    uint32_t n_spec = 0, n_srec = 0;
    // block-strided so that the block reserves its output slots together
    for (uint32_t bbase = blockIdx.x * kShadeBlock; bbase < count; bbase += gridDim.x * kShadeBlock) {
        const uint32_t i = bbase + threadIdx.x;
        const bool active = i < count;
        uint32_t aux = 0, pix = 0, smp = 0;
        int32_t tri = -1;
        int kind = -1;            // 0 miss, 1 Lambert, 2 glass, 3 bubbly glass (both queued)
        bool want_shadow = false, keep = false, spec = false, gray = false;
        V3<R> x = {R(0), R(0), R(0)}, dnew = x, nrm = x;
        R cs = R(0), g = R(0), rho_g = R(1);
        int mat = 0;
        const JobDev *jb = nullptr;
        BandDev bd = {0, 0, 0, 0};
        if (active) {
            const PathS<R> ps = rec_load(Pi.s + i);
            aux = ps.aux;
            pix = ps.pix;
            smp = ps.smp;
            spec = (smp & kSpectral) != 0u;
            g = ps.g;
            const int depth = (int)(aux & 0xffu);
            jb = &jobs[kOne ? 0u : aux >> kAuxJobShift];
            bd = bands[(aux >> kAuxBandShift) & ((1u << kAuxBandBits) - 1u)];
            const HitRec<R> hr = rec_load(w.hit + i);
            tri = hr.tri;
            const bool last = depth >= jb->max_depth - 1;
            if (tri < 0) {
                kind = 0;
            } else {
                const TriDev tr = load_tri(jb->sc.tris, tri);
                mat = __float_as_int(tr.b.w);
                const int mt = __float_as_int(tr.c.w);
                if (mt == 0 || mt == 3) {
                    kind = 1;
                    gray = mt == 3;
                    if (gray) rho_g = gld((const R *)jb->rho + (size_t)mat * jb->ms + bd.l0);
                    const PathO<R> po = rec_load(Pi.o + i);
                    const PathD<R> pd = rec_load(Pi.d + i);
                    const V3<R> o = {po.x, po.y, po.z}, d = {pd.x, pd.y, pd.z};
                    x = o + hr.t * d;
                    const V3<R> ng = tri_normal<R>(tr);
                    const V3<R> ns = dot(ng, d) > R(0) ? R(-1) * ng : ng;
                    const V3<R> sun = {R(jb->sc.sun[0]), R(jb->sc.sun[1]), R(jb->sc.sun[2])};
                    cs = dot(ns, sun);
                    // with the caustic map, every Lambert vertex keeps a record for
                    // its gather (the sun's term is zero where it faces away)
                    want_shadow = cs > R(0) || jb->caustic;
                    nrm = ns;
                    keep = !last;
                    if (!last) {
                        const uint4 rr = vertex_draws(jb->seed, jb->job_word, pix, smp & ~kSpectral, depth, 0);
                        dnew = cosine_dir(ns, u01<R>(rr.y), u01<R>(rr.z));
                    }
                } else if (!last) {
                    // no light sum at glass; a glass vertex at the depth limit ends the path
                    kind = mt == 2 ? 3 : 2;
                    if (kind == 2) {   // gathered for the glass pass's record (cs and rho_g,
                                       // unused at glass, carry the barycentrics)
                        const PathO<R> po = rec_load(Pi.o + i);
                        const PathD<R> pd = rec_load(Pi.d + i);
                        dnew = {pd.x, pd.y, pd.z};
                        x = V3<R>{po.x, po.y, po.z} + hr.t * dnew;
                        cs = hr.u;
                        rho_g = hr.v;
                    }
                }
            }
        }
        n_spec += (uint32_t)__popcll(__ballot(active && spec));   // wave-uniform counts
        // glass and bubbly queues, shadow and sky records, pool slots: one
        // atomic per block and buffer
        const bool want[5] = {kind == 2, kind == 3, want_shadow, keep, kind == 0};
        uint32_t *const ctr[5] = {&w.cnt->gcount, &w.cnt->bcount, &w.cnt->scount, &w.cnt->count[cur ^ 1],
                                  &w.cnt->kcount};
        uint32_t slot[5];
        block_reserve<5, kShadeBlock / 64>(want, ctr, slot, s_cnt, s_base);
        if (kind == 2) {
            GlassRec<R> r;
            r.x[0] = x.x; r.x[1] = x.y; r.x[2] = x.z;
            r.d[0] = dnew.x; r.d[1] = dnew.y; r.d[2] = dnew.z;
            r.g = g; r.u = cs; r.v = rho_g;
            r.tri = tri; r.aux = aux; r.pix = pix; r.smp = smp; r.slot = i;
            rec_store(w.grec + slot[0], r);
        }
        if (kind == 3) w.gidx[w.cap - 1u - slot[1]] = i;
        uint32_t sslot = slot[2];
        if (want_shadow && sslot >= w.cap) { w.cnt->overflow |= 1u; want_shadow = false; }
        uint32_t om = slot[3];
        if (keep && om >= w.cap) { w.cnt->overflow |= 1u; keep = false; }
        // row tasks: flags, record row, albedo row offset (see below)
        uint32_t rflags = 0, rrec = 0, rrho = 0;
        R gn = g;
        if (kind == 1) {
            // Lambert: the shadow record carries g rho cos / pi (rho when gray), the
            // continuing path g rho; a spectral albedo or spectral weights keep
            // per-wavelength factors
            const bool out_spec = spec || !gray;
            const R thr = R(jb->beta_thr);
            if (gray) gn = g * rho_g;
            if (want_shadow) {
                w.sx[sslot] = x.x; w.sy[sslot] = x.y; w.sz[sslot] = x.z;
                w.sskip[sslot] = tri;
                w.spix[sslot] = pix | (out_spec ? kSpectral : 0u);
                w.saux[sslot] = aux;
                w.scs[sslot] = cs > R(0) ? gn * inv_pi * cs : R(0);
                if (jb->caustic) {
                    w.sgr[sslot] = gn * inv_pi;
                    w.snx[sslot] = nrm.x; w.sny[sslot] = nrm.y; w.snz[sslot] = nrm.z;
                }
            }
            if (keep) {
                // the energy threshold of a gray path acts on g
                put_path<R>(Po, om, x, dnew, tri, pix, (smp & ~kSpectral) | (out_spec ? kSpectral : 0u), aux + 1u,
                            (!out_spec && gn < thr) ? R(0) : gn);
            }
            if (out_spec) {
                rflags = (spec ? kRowSrc : 0u) | (gray ? 0u : kRowRho) | (want_shadow ? kRowRec : 0u) |
                         (keep ? kRowKeep : 0u);
                rrec = sslot;
                rrho = (uint32_t)(mat * jb->ms + bd.l0);
            }
        }
        // escaping paths: a sky record each (summed per pixel by the
        // accumulation pass, which keeps its waves dense)
        const uint32_t kslot = slot[4];
        if (kind == 0 && kslot >= w.cap) w.cnt->overflow |= 1u;   // cannot happen: one record per path
        if (kind == 0 && kslot < w.cap) {
            const uint32_t r = w.cap - 1u - kslot;
            w.spix[r] = pix | (spec ? kSpectral : 0u);
            w.saux[r] = aux;
            w.scs[r] = g;
            if (spec) {
                rflags = kRowSrc | kRowRec;
                rrec = r;
            }
        }
        // Per-wavelength rows (16-byte aligned, padded to a multiple of 4; the
        // padding is unused): the factors (or 1), times the albedo row for a
        // spectral albedo, go to the record and, thresholded, to the
        // continuing path.
        n_srec += (uint32_t)__popcll(__ballot((rflags & kRowRec) != 0u));
        if (!(rflags & (kRowRec | kRowKeep))) rflags = 0;
        if (rflags) rflags |= (uint32_t)bd.nb << kRowNbShift | ((bd.l0 & 3) == 0 ? kRowAl : 0u);
        const RowTasks rt = row_tasks(rflags != 0, nbm, s_map);
        for (int b0 = 0; b0 < rt.n; b0 += rt.ng) {
            const int src = rt.src(b0, s_map);
            const uint32_t f = (uint32_t)__shfl((int)rflags, src);
            const uint32_t si = (uint32_t)__shfl((int)i, src), rec = (uint32_t)__shfl((int)rrec, src);
            const uint32_t so = (uint32_t)__shfl((int)om, src), ro = (uint32_t)__shfl((int)rrho, src);
            const R sg = __shfl(gn, src);
            const uint32_t sjob = kOne ? 0u : (uint32_t)__shfl((int)(aux >> kAuxJobShift), src);
            const int nb = (int)(f >> kRowNbShift), j = rt.j;
            if (!rt.busy(b0) || j >= nb) continue;
            Vec4<R> v;
            if (f & kRowSrc) v = row_load4(Pi.beta + aosoa(si, j, nbm));
            else v.v[0] = v.v[1] = v.v[2] = v.v[3] = R(1);
            const JobDev *sj = &jobs[sjob];
            if (f & kRowRho) {
                const Vec4<R> r4 = tab4((const R *)sj->rho + ro, (f & kRowAl) != 0u, j, nb);
#pragma unroll
                for (int q = 0; q < 4; ++q) v.v[q] *= r4.v[q];
            }
            if (f & kRowRec) row_store4(w.contrib + aosoa(rec, j, nbm), v);
            if (f & kRowKeep) {
                const R thr = R(sj->beta_thr);
#pragma unroll
                for (int q = 0; q < 4; ++q) v.v[q] = (sg * v.v[q] < thr) ? R(0) : v.v[q];
                row_store4(Po.beta + aosoa(so, j, nbm), v);
            }
        }
    }
    if (lane == 0 && (n_spec | n_srec)) {
        atomicAdd(&w.cnt->spec_paths, (unsigned long long)n_spec);
        atomicAdd(&w.cnt->spec_records, (unsigned long long)n_srec);
    }
}

// ---------------------------------------------------------------------------
// Outputs of a split vertex: the kept path (direction dnew, the wavelengths
// whose reflect bit is clear, or all of them when there is no fork) and, when
// both branches occur, a forked path (direction drefl, the wavelengths whose
// bit is set).  The new per-wavelength factors sit in Pi.beta at slot i; both
// outputs keep the scalar factor g.  Called by every thread of the block
// (block-uniform loop); one reservation per block.
template <class R>
__device__ __forceinline__ void emit_paths(const Work<R> &w, const Pool<R> &Po, int cur, bool &keep, bool &fork,
                                           V3<R> x, V3<R> dnew, V3<R> drefl, uint32_t pix, uint32_t smp, uint32_t aux,
                                           int32_t tri, R g, uint32_t &om, uint32_t &of, uint32_t *s_cnt,
                                           uint32_t *s_base)
{
    smp |= kSpectral;   // the outputs carry per-wavelength factors
    const bool want[2] = {keep, fork};
    uint32_t *const ctr[2] = {&w.cnt->count[cur ^ 1], &w.cnt->count[cur ^ 1]};
    uint32_t slot[2];
    block_reserve<2>(want, ctr, slot, s_cnt, s_base);
    om = slot[0];
    of = slot[1];
    if (keep && om >= w.cap) { w.cnt->overflow |= 1u; keep = false; }
    if (fork && of >= w.cap) { w.cnt->overflow |= 1u; fork = false; }
    if (keep) put_path<R>(Po, om, x, dnew, tri, pix, smp, aux + 1u, g);
    if (fork) put_path<R>(Po, of, x, drefl, tri, pix, smp, aux + 1u, g);
}

// ---------------------------------------------------------------------------
// Glass vertices (thin slab, Sec. 6 thickness map): per wavelength the path
// reflects with probability R/(R+T) and otherwise passes straight through,
// its weight multiplied by R + T.  When a band splits, the path forks: the
// reflected wavelengths continue in a new pool slot.
// ---------------------------------------------------------------------------
template <class R, bool kOne>
__global__ void __launch_bounds__(kBlock) k_shade_glass(const JobDev *__restrict__ jobs, const BandDev *__restrict__ bands, Work<R> w, int cur)
{
    const uint32_t count = min(w.cnt->gcount, w.cap);
    const Pool<R> Pi = w.p[cur], Po = w.p[cur ^ 1];
    const int nbm = w.nbmax;
    const uint32_t lane = lane_id();
    __shared__ uint32_t s_cnt[(kBlock / 64) * 2], s_base[2];
    __shared__ uint32_t s_map_all[kBlock];
    uint32_t *const s_map = s_map_all + (threadIdx.x & ~63u);
    uint32_t n_fork = 0, n_in = 0, n_spec = 0;
    // block-strided: the block reserves its output slots together
    for (uint32_t base = blockIdx.x * kBlock; base < count; base += gridDim.x * kBlock) {
        const bool active = base + threadIdx.x < count;
        n_in += active ? 1u : 0u;
        uint32_t i = 0, aux = 0, pix = 0, smp = 0, flags = 0, mo = 0;
        int32_t tri = -1;
        V3<R> x = {R(0), R(0), R(0)}, dnew = x, drefl = x;
        R g = R(0), cos_i = R(0), thick = R(0), u0 = R(0);
        if (active) {
            const GlassRec<R> gr = rec_load(w.grec + base + threadIdx.x);
            i = gr.slot;
            aux = gr.aux;
            pix = gr.pix;
            smp = gr.smp;
            const bool spec = (smp & kSpectral) != 0u;
            n_spec += spec ? 1u : 0u;
            g = gr.g;
            const int depth = (int)(aux & 0xffu);
            const JobDev *jb = &jobs[kOne ? 0u : aux >> kAuxJobShift];
            const BandDev bd = bands[(aux >> kAuxBandShift) & ((1u << kAuxBandBits) - 1u)];
            tri = gr.tri;
            const V3<R> d = {gr.d[0], gr.d[1], gr.d[2]};
            x = {gr.x[0], gr.x[1], gr.x[2]};
            const TriDev tr = load_tri(jb->sc.tris, tri);
            const int mat = __float_as_int(tr.b.w);
            const V3<R> ng = tri_normal<R>(tr);
            const uint4 rr = vertex_draws(jb->seed, jb->job_word, pix, smp & ~kSpectral, depth, 0);
            u0 = u01<R>(rr.x);
            cos_i = fabs(dot(d, ng));
            int me;
            pane_at<R>(jb->sc, tri, mat, gr.u, gr.v, me, thick);
            dnew = d;
            drefl = d - (R(2) * dot(d, ng)) * ng;
            flags = (spec ? kRowSrc : 0u) | ((bd.l0 & 3) == 0 ? kRowAl : 0u) | (uint32_t)bd.nb << kRowNbShift |
                    (uint32_t)bd.l0 << 16;
            mo = (uint32_t)(me * jb->ms + bd.l0);
        }
        // Per wavelength: the new factor b (R + T) goes back to the input
        // slot's row (a path without per-wavelength factors gets them here),
        // negated where the wavelength reflects; the padding is set to zero.
        // The wave takes the rows together (see RowTasks).
        const RowTasks rt = row_tasks(active, nbm, s_map);
        bool anyR = false, anyT = false;
        for (int b0 = 0; b0 < rt.n; b0 += rt.ng) {
            const int src = rt.src(b0, s_map);
            const uint32_t f = (uint32_t)__shfl((int)flags, src);
            const uint32_t si = (uint32_t)__shfl((int)i, src), smo = (uint32_t)__shfl((int)mo, src);
            const R sc = __shfl(cos_i, src), st = __shfl(thick, src), su = __shfl(u0, src), sg = __shfl(g, src);
            const uint32_t sjob = kOne ? 0u : (uint32_t)__shfl((int)(aux >> kAuxJobShift), src);
            const int nb = (int)((f >> kRowNbShift) & 0xffu), j = rt.j;
            bool lR = false, lT = false;
            if (rt.busy(b0) && j < nb) {
                const JobDev *sj = &jobs[sjob];
                const bool al = (f & kRowAl) != 0u;
                R *__restrict__ brow = Pi.beta + aosoa(si, 0, nbm);
                Vec4<R> b4;
                if (f & kRowSrc) b4 = row_load4(brow + j);
                else b4.v[0] = b4.v[1] = b4.v[2] = b4.v[3] = R(1);
                const Vec4<R> l4 = tab4((const R *)sj->lam + (f >> 16), al, j, nb),
                              n4 = tab4((const R *)sj->n + smo, al, j, nb),
                              k4 = tab4((const R *)sj->k + smo, al, j, nb),
                              t4 = tab4((const R *)sj->tint + smo, al, j, nb);
                const R thr = R(sj->beta_thr);
                Vec4<R> o4;
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    o4.v[q] = R(0);
                    if (j + q >= nb || b4.v[q] == R(0)) continue;
                    R Rr, Tt;
                    slab_RT<R>(sc, l4.v[q], st, n4.v[q], k4.v[q], t4.v[q], Rr, Tt);
                    const R rtot = Rr + Tt;
                    R bn = b4.v[q] * rtot;
                    if (sg * bn < thr) bn = R(0);
                    if (bn == R(0)) continue;
                    if (rtot > R(0) && su < Rr / rtot) {
                        lR = true;
                        o4.v[q] = -bn;
                    } else {
                        lT = true;
                        o4.v[q] = bn;
                    }
                }
                row_store4(brow + j, o4);
            }
            const uint64_t bR = __ballot(lR), bT = __ballot(lT);
            uint64_t mine;
            if (rt.mine(active, b0, mine)) {
                anyR = (bR & mine) != 0u;
                anyT = (bT & mine) != 0u;
            }
        }
        bool keep = anyR || anyT, fork = anyR && anyT;
        if (anyR && !anyT) dnew = drefl;
        n_fork += fork ? 1u : 0u;
        uint32_t om, of;
        emit_paths<R>(w, Po, cur, keep, fork, x, dnew, drefl, pix, smp, aux, tri, g, om, of, s_cnt, s_base);
        // the rows of the outputs: the kept path takes the transmitted
        // wavelengths (all of them without a fork), the forked path the
        // reflected ones; the same lanes read the elements they wrote above
        const uint32_t ef = flags | (keep ? kRowKeep : 0u) | (fork ? kRowFork : 0u);
        for (int b0 = 0; b0 < rt.n; b0 += rt.ng) {
            const int src = rt.src(b0, s_map);
            const uint32_t f = (uint32_t)__shfl((int)ef, src);
            const uint32_t si = (uint32_t)__shfl((int)i, src), so = (uint32_t)__shfl((int)om, src),
                           sf = (uint32_t)__shfl((int)of, src);
            const int nb = (int)((f >> kRowNbShift) & 0xffu), j = rt.j;
            if (!rt.busy(b0) || j >= nb || !(f & kRowKeep)) continue;
            const bool fk = (f & kRowFork) != 0u;
            const Vec4<R> b = row_load4(Pi.beta + aosoa(si, j, nbm));
            Vec4<R> k4, f4;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const bool refl = signbit(b.v[q]);
                const R a = fabs(b.v[q]);
                k4.v[q] = (fk && refl) ? R(0) : a;
                f4.v[q] = refl ? a : R(0);
            }
            row_store4(Po.beta + aosoa(so, j, nbm), k4);
            if (fk) row_store4(Po.beta + aosoa(sf, j, nbm), f4);
        }
    }
    for (int off = 32; off > 0; off >>= 1) {
        n_fork += __shfl_xor(n_fork, off);
        n_in += __shfl_xor(n_in, off);
        n_spec += __shfl_xor(n_spec, off);
    }
    if (lane == 0 && n_fork) atomicAdd(&w.cnt->forks, (unsigned long long)n_fork);
    if (lane == 0 && n_in) atomicAdd(&w.cnt->glass[0], (unsigned long long)n_in);
    if (lane == 0 && n_spec) atomicAdd(&w.cnt->glass[1], (unsigned long long)n_spec);
}

// ---------------------------------------------------------------------------
// Bubbly panes (air micro-particles in the glass, Sec. 1; volume scattering,
// Sec. 6).  A vertex is evaluated by the exact walk or by the surrogate
// network; the fallback mode takes the walk where the error table flags the
// vertex's cell.
// ---------------------------------------------------------------------------
struct BubblyVertex {
    uint32_t i;                 // pool slot
    const JobDev *jb;
    BandDev bd;
    int32_t tri, mat, pane;
    int mode;                   // kBtdfExact or kBtdfSurrogate after the table check
    double sigma, n_ref, rho;
};

template <class R>
__device__ __forceinline__ BubblyVertex bubbly_vertex(const JobDev *jobs, const BandDev *bands, const Work<R> &w,
                                                      const Pool<R> &Pi, uint32_t e, V3<R> &d, V3<R> &ng, R &cos_i,
                                                      R &thick)
{
    BubblyVertex v;
    v.i = w.gidx[w.cap - 1u - e];
    const uint32_t aux = rec_load(Pi.s + v.i).aux;
    v.jb = &jobs[aux >> kAuxJobShift];
    v.bd = bands[(aux >> kAuxBandShift) & ((1u << kAuxBandBits) - 1u)];
    const HitRec<R> hr = rec_load(w.hit + v.i);
    v.tri = hr.tri;
    const TriDev tr = load_tri(v.jb->sc.tris, v.tri);
    v.mat = __float_as_int(tr.b.w);
    const PathD<R> pd = rec_load(Pi.d + v.i);
    d = {pd.x, pd.y, pd.z};
    ng = tri_normal<R>(tr);
    cos_i = fabs(dot(d, ng));
    thick = pane_thickness<R>(v.jb->sc, v.tri, v.mat, hr.u, hr.v);
    const double *b = v.jb->sc.mat_bub + 4 * (size_t)v.mat;
    v.sigma = gld(b);
    v.n_ref = gld(b + 1);
    v.rho = gld(b + 2);
    v.pane = (int)gld(b + 3);
    v.mode = v.jb->btdf_mode;
    if (v.mode == kBtdfFallback) {
        const int c = err_cell<R>(v.jb->err_dims, v.pane, cos_i, thick, R(v.rho));
        v.mode = gld(v.jb->err_table + c) > v.jb->err_bound ? kBtdfExact : kBtdfSurrogate;
    }
    return v;
}

// Surrogate at the bubbly vertices: for each vertex the network's (R, T) at
// every wavelength of its band and its lobe width w at kLambdaRef.  The
// weights are multiplied by R + T in place; R / (R + T) and w are kept for
// k_shade_bubbly.
//
// FP32 build, on the matrix cores (BF16 operands, FP32 sums).  A wave takes
// 64 vertices, sets them up one per lane (the chain of dependent loads of a
// vertex runs in parallel across the lanes) into LDS records, then runs each
// vertex's band wavelengths (and the reference one) through the network 16
// at a time.  Each layer is H' = W H^T on 16x16x32 tiles: the 16 samples are
// the columns, so a lane ends a layer holding, for its sample c = lane % 16,
// the outputs 16 t + 4 g + r (g = lane / 16, r = 0..3) of each output tile
// t.  Those are exactly the operand rows the next layer needs if its input
// index k = 32 s + 8 g + i (K step s, i = 0..7) stands for the previous
// layer's output 16 (2 s + i / 4) + 4 g + i % 4: the layers' weight columns
// are gathered in that order, and activations never leave the registers.
// Every lane holds the A fragments of all four layers (W1 4, W2 8, W3 8, W4
// 2 tiles of 8 BF16) for the whole launch; the biases enter as the
// accumulators' initial values.  Layer 1 has 12 inputs and runs on the
// 16x16x16 form (input k = 4 g + i).  Two tiles go through the layers
// together, so each layer has eight independent products in flight.  The
// three outputs of each sample go to LDS, and the heads and the weight
// updates then run once per vertex over all 64 lanes.
constexpr int kEvalBlock = 256;
constexpr int kEvalMaxTiles = ((kMaxBand + 1 + 15) / 16 + 1) / 2 * 2;   // tiles run in pairs

__device__ __forceinline__ int eval_in(int s, int g, int i)   // previous-layer output behind input k
{
    return 16 * (2 * s + (i >> 2)) + 4 * g + (i & 3);
}

typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef float f32x2 __attribute__((ext_vector_type(2)));
typedef short s16x2 __attribute__((ext_vector_type(2)));

// relu(a), relu(b) rounded to BF16 and packed in one word.  A BF16 with its
// sign bit set is a negative 16-bit integer, so the integer maximum with 0
// after the rounding is the relu (and clears -0).
__device__ __forceinline__ uint32_t pk_relu_bf16(float a, float b)
{
    const s16x2 h = __builtin_bit_cast(s16x2, __builtin_convertvector((f32x2){a, b}, bf16x2));
    return __builtin_bit_cast(uint32_t, __builtin_elementwise_max(h, (s16x2)0));
}

// A vertex as the evaluation needs it: its pool slot, pane, band size, mode
// and spectral flag, the wavelength-independent features and its band's
// wavelength row.
struct EvalRec {
    uint32_t i, pane, nb, flags;   // flags: 1 surrogate, 2 spectral weights
    float f0, f2, f3;              // cos, (d - 3.5) / 1.5, rho / 34
    uint32_t pad;
    const void *lam;
};

template <class R>
__global__ void __launch_bounds__(kEvalBlock) __attribute__((amdgpu_waves_per_eu(3))) k_bubbly_eval_mfma(const JobDev *__restrict__ jobs,
                                                                const BandDev *__restrict__ bands, Work<R> w,
                                                                int cur, const float *__restrict__ P,
                                                                const float *__restrict__ E, int n_panes)
{
    constexpr int kW = kEvalBlock / 64, kS = kEvalMaxTiles * 16;
    __shared__ f32x4 s_bias[49];   // b1 b2 b3 as 16 f32x4 each, then b4 padded
    __shared__ float s_E[kMaxPanes * 8];
    __shared__ EvalRec s_rec[kW][64];
    __shared__ float s_lam[kW][kS];      // wavelength feature (lambda - 580) / 200 of sample j
    __shared__ float s_out[kW][3][kS];
    for (int i = threadIdx.x; i < 49; i += blockDim.x) {
        const int layer = i >> 4, q = i & 15;
        const int off = layer == 0 ? kOffB1 : layer == 1 ? kOffB2 : layer == 2 ? kOffB3 : kOffB4;
        f32x4 v;
        for (int r = 0; r < 4; ++r) v[r] = (layer == 3 && r >= 3) ? 0.0f : gld(P + off + 4 * q + r);
        s_bias[i] = v;
    }
    for (int i = threadIdx.x; i < 8 * min(n_panes, kMaxPanes); i += blockDim.x) s_E[i] = gld(E + i);
    __syncthreads();
    const int l = (int)lane_id(), g = l >> 4, c = l & 15, wv = (int)(threadIdx.x >> 6);
    float(*so)[kS] = s_out[wv];
    float *sl = s_lam[wv];
    // A fragments: lane (g, c) holds row c of each output tile and the
    // inputs of its K slice
    s16x4 A1[4];
    bf16x8 A2[4][2], A3[4][2], A4[2];
    for (int t = 0; t < 4; ++t) {
        for (int i = 0; i < 4; ++i) {
            const int k = 4 * g + i;
            A1[t][i] = bits((__bf16)(k < 12 ? gld(P + kOffW1 + (16 * t + c) * 12 + k) : 0.0f));
        }
        for (int s = 0; s < 2; ++s)
            for (int i = 0; i < 8; ++i) {
                const int k = eval_in(s, g, i);
                A2[t][s][i] = (__bf16)gld(P + kOffW2 + (16 * t + c) * 64 + k);
                A3[t][s][i] = (__bf16)gld(P + kOffW3 + (16 * t + c) * 64 + k);
            }
    }
    for (int s = 0; s < 2; ++s)
        for (int i = 0; i < 8; ++i)
            A4[s][i] = (__bf16)(c < 3 ? gld(P + kOffW4 + c * 64 + eval_in(s, g, i)) : 0.0f);

    const Pool<R> Pi = w.p[cur];
    const uint32_t stride = (uint32_t)w.nbmax + 1u;          // band wavelengths + the reference one
    const uint32_t per_v = ((stride + 15u) / 16u + 1u) & ~1u;   // tiles per vertex, even
    const uint32_t nv = min(w.cnt->bcount, w.cap);
    const uint32_t wave = (blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const uint32_t nw = (gridDim.x * blockDim.x) >> 6;
    const void *lam_cached = nullptr;
    uint32_t nb_cached = 0;
    for (uint32_t base = wave * 64u; base < nv; base += nw * 64u) {
        {
            EvalRec rc{};
            const uint32_t e = base + (uint32_t)l;
            if (e < nv) {
                V3<R> d, ng;
                R cos_i, thick;
                const BubblyVertex v = bubbly_vertex<R>(jobs, bands, w, Pi, e, d, ng, cos_i, thick);
                if (v.mode == kBtdfSurrogate) {
                    rc.i = v.i;
                    rc.pane = (uint32_t)v.pane;
                    rc.nb = (uint32_t)v.bd.nb;
                    rc.flags = 1u | ((rec_load(Pi.s + v.i).smp & kSpectral) ? 2u : 0u);
                    rc.f0 = (float)cos_i;
                    rc.f2 = ((float)thick - 3.5f) / 1.5f;
                    rc.f3 = (float)v.rho / 34.0f;
                    rc.lam = (const R *)v.jb->lam + v.bd.l0;
                }
            }
            s_rec[wv][l] = rc;
        }
        wave_sync();
        const uint32_t nk = min(64u, nv - base);
        for (uint32_t k = 0; k < nk; ++k) {
            const EvalRec r = s_rec[wv][k];   // the same for every lane
            if (!(r.flags & 1u)) continue;
            // the weights this vertex scales, fetched while the network runs
            R bq[(kS + 63) / 64];
            for (int q = 0; q < (kS + 63) / 64; ++q) {
                const uint32_t j = (uint32_t)(l + 64 * q);
                bq[q] = ((r.flags & 2u) && j < r.nb) ? Pi.beta[aosoa(r.i, (int)j, w.nbmax)] : R(1);
            }
            if (r.lam != lam_cached || r.nb != nb_cached) {   // most vertices share a band
                for (uint32_t j = (uint32_t)l; j < per_v * 16u; j += 64u)
                    sl[j] = ((j < r.nb ? (float)gld((const R *)r.lam + j) : kLambdaRef) - 580.0f) * 0.005f;
                lam_cached = r.lam;
                nb_cached = r.nb;
                wave_sync();
            }
            // layer-1 operand of sample c: features 4 g .. 4 g + 3; only the
            // wavelength (feature 1) changes from tile to tile
            s16x4 x0;
            {
                const float *Ep = s_E + 8 * r.pane;
                float f[4];
                if (g == 0) {
                    f[0] = r.f0;
                    f[1] = 0.0f;
                    f[2] = r.f2;
                    f[3] = r.f3;
                } else {
                    for (int i = 0; i < 4; ++i) f[i] = g < 3 ? Ep[4 * (g - 1) + i] : 0.0f;
                }
                for (int i = 0; i < 4; ++i) x0[i] = bits((__bf16)f[i]);
            }
            for (uint32_t tile = 0; tile < per_v; tile += 2u) {
                s16x4 x[2];
                for (int u = 0; u < 2; ++u) {
                    x[u] = x0;
                    if (g == 0) x[u][1] = bits((__bf16)sl[(tile + u) * 16u + (uint32_t)c]);
                }
                bf16x8 H[2][2];
                f32x4 acc[2][4];
                auto epilogue = [&]() {
                    for (int u = 0; u < 2; ++u)
                        for (int s = 0; s < 2; ++s) {
                            uint4 q;
                            q.x = pk_relu_bf16(acc[u][2 * s][0], acc[u][2 * s][1]);
                            q.y = pk_relu_bf16(acc[u][2 * s][2], acc[u][2 * s][3]);
                            q.z = pk_relu_bf16(acc[u][2 * s + 1][0], acc[u][2 * s + 1][1]);
                            q.w = pk_relu_bf16(acc[u][2 * s + 1][2], acc[u][2 * s + 1][3]);
                            H[u][s] = __builtin_bit_cast(bf16x8, q);
                        }
                };
                // the biases are read from LDS at each use rather than held
                // in registers across the loop
                int z = 0;
                asm volatile("" : "+v"(z));
                const f32x4 *sb = s_bias + z;
                for (int t = 0; t < 4; ++t)
                    for (int u = 0; u < 2; ++u) acc[u][t] = mfma16(A1[t], x[u], sb[4 * t + g]);
                epilogue();
                for (int t = 0; t < 4; ++t)
                    for (int u = 0; u < 2; ++u)
                        acc[u][t] = mfma32(A2[t][1], H[u][1], mfma32(A2[t][0], H[u][0], sb[16 + 4 * t + g]));
                epilogue();
                for (int t = 0; t < 4; ++t)
                    for (int u = 0; u < 2; ++u)
                        acc[u][t] = mfma32(A3[t][1], H[u][1], mfma32(A3[t][0], H[u][0], sb[32 + 4 * t + g]));
                epilogue();
                for (int u = 0; u < 2; ++u) {
                    const f32x4 o = mfma32(A4[1], H[u][1], mfma32(A4[0], H[u][0], sb[48]));
                    // outputs 0..2 of sample c sit in lanes g = 0
                    if (g == 0)
                        for (int q = 0; q < 3; ++q) so[q][(tile + u) * 16u + (uint32_t)c] = o[q];
                }
            }
            wave_sync();
            for (int q = 0; q < (kS + 63) / 64; ++q) {
                const uint32_t j = (uint32_t)(l + 64 * q);
                const bool ref = j == stride - 1u;
                if (!(j < r.nb || ref)) continue;
                float Rr, Tt, wl;
                heads(so[0][j], so[1][j], so[2][j], Rr, Tt, wl);
                if (ref) {
                    w.bw[r.i] = R(wl);
                } else {
                    const size_t a = aosoa(r.i, (int)j, w.nbmax);
                    Pi.beta[a] = bq[q] * R(Rr + Tt);
                    w.bratio[a] = R(Rr / (Rr + Tt));
                }
            }
            wave_sync();
        }
    }
}

// FP64 build: the same network evaluated in double, one tuple per thread
// (the arithmetic of the FP64 reference network).
__device__ double net_fp64(const float *p, const float *E, int pane, double cos_i, double lam, double d, double rho,
                           double out[3])
{
    double x[12], h1[64], h2[64];
    x[0] = cos_i;
    x[1] = (lam - 580.0) / 200.0;
    x[2] = (d - 3.5) / 1.5;
    x[3] = rho / 34.0;
    for (int e = 0; e < 8; ++e) x[4 + e] = (double)E[8 * pane + e];
    const float *W1 = p, *b1 = p + 768, *W2 = p + 832, *b2 = p + 4928, *W3 = p + 4992, *b3 = p + 9088,
                *W4 = p + 9152, *b4 = p + 9344;
    for (int o = 0; o < 64; ++o) {
        double s = b1[o];
        for (int i = 0; i < 12; ++i) s += (double)W1[o * 12 + i] * x[i];
        h1[o] = s > 0.0 ? s : 0.0;
    }
    for (int o = 0; o < 64; ++o) {
        double s = b2[o];
        for (int i = 0; i < 64; ++i) s += (double)W2[o * 64 + i] * h1[i];
        h2[o] = s > 0.0 ? s : 0.0;
    }
    for (int o = 0; o < 64; ++o) {
        double s = b3[o];
        for (int i = 0; i < 64; ++i) s += (double)W3[o * 64 + i] * h2[i];
        h1[o] = s > 0.0 ? s : 0.0;   // h3
    }
    double o3[3];
    for (int o = 0; o < 3; ++o) {
        double s = b4[o];
        for (int i = 0; i < 64; ++i) s += (double)W4[o * 64 + i] * h1[i];
        o3[o] = s;
    }
    const double m = fmax(fmax(o3[0], o3[1]), 0.0);
    const double a = exp(o3[0] - m), b = exp(o3[1] - m), c = exp(-m);
    out[0] = a / (a + b + c);
    out[1] = b / (a + b + c);
    out[2] = o3[2] > 30.0 ? o3[2] : log1p(exp(o3[2]));
    return out[0];
}

__global__ void __launch_bounds__(kBlock) k_bubbly_eval_fp64(const JobDev *__restrict__ jobs, const BandDev *__restrict__ bands, Work<double> w,
                                                            int cur, const float *params, const float *E)
{
    const Pool<double> Pi = w.p[cur];
    const uint32_t stride = (uint32_t)w.nbmax + 1u;
    const uint64_t ntup = (uint64_t)min(w.cnt->bcount, w.cap) * stride;
    for (uint64_t tu = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; tu < ntup;
         tu += (uint64_t)gridDim.x * blockDim.x) {
        const uint32_t e = (uint32_t)(tu / stride), j = (uint32_t)(tu % stride);
        V3<double> d, ng;
        double cos_i, thick;
        const BubblyVertex v = bubbly_vertex<double>(jobs, bands, w, Pi, e, d, ng, cos_i, thick);
        if (v.mode != kBtdfSurrogate || (j >= (uint32_t)v.bd.nb && j != stride - 1u)) continue;
        const double lam = j == stride - 1u ? (double)kLambdaRef : gld((const double *)v.jb->lam + v.bd.l0 + j);
        double y[3];
        net_fp64(params, E, v.pane, cos_i, lam, thick, v.rho, y);
        if (j == stride - 1u) {
            w.bw[v.i] = y[2];
        } else {
            const size_t q = aosoa(v.i, (int)j, w.nbmax);
            const double b = (rec_load(Pi.s + v.i).smp & kSpectral) ? Pi.beta[q] : 1.0;
            Pi.beta[q] = b * (y[0] + y[1]);
            w.bratio[q] = y[0] / (y[0] + y[1]);
        }
    }
}

// Bubbly vertex shading.  Exact walk: the entry interface decides per
// wavelength (complex index, shared draw); the wavelengths that enter share
// one walk inside (the pane's index at kLambdaRef) and are weighted by
// exp(-alpha L).  Surrogate: reflect where u0 < R / (R + T), else the
// transmitted lobe of width w, folded onto the far side of the pane.  Either
// way a band splits into at most a reflected and a continuing packet.
//
// One lane per vertex for the set-up and the walk; the per-wavelength rows
// (weights, surrogate ratios, tables) are taken by the whole wave (see
// RowTasks), with a row's weights written back signed: negative where the
// wavelength reflects.  Exact vertices take two row passes around the walk
// (the entry decisions, which tell whether the walk is needed, then the
// weights after it); surrogate vertices one.
constexpr uint32_t kRowExact = 64u;

// FP32: four waves per SIMD (the walk is latency-bound)
template <class R>
__global__ void __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(sizeof(R) == 4 ? 4 : 1))) k_shade_bubbly(const JobDev *__restrict__ jobs, const BandDev *__restrict__ bands, Work<R> w, int cur)
{
    const uint32_t count = min(w.cnt->bcount, w.cap);
    if (blockIdx.x == 0 && threadIdx.x == 0) w.cnt->bubbly += count;
    const Pool<R> Pi = w.p[cur], Po = w.p[cur ^ 1];
    const int nbm = w.nbmax;
    const uint32_t lane = lane_id();
    __shared__ uint32_t s_cnt[(kBlock / 64) * 2], s_base[2];
    __shared__ uint32_t s_map_all[kBlock];
    uint32_t *const s_map = s_map_all + (threadIdx.x & ~63u);
    uint32_t n_fork = 0;
    // block-strided: the block reserves its output slots together
    for (uint32_t base = blockIdx.x * kBlock; base < count; base += gridDim.x * kBlock) {
        const bool active = base + threadIdx.x < count;
        uint32_t i = 0, aux = 0, pix = 0, smp = 0, flags = 0, mo = 0;
        int32_t tri = -1;
        V3<R> x = {R(0), R(0), R(0)}, dnew = x, d = x, ng = x;
        R g = R(0), cos_i = R(0), thick = R(0), u0 = R(0), sigma = R(0), n_ref = R(0);
        int pol = 0;
        WalkStream ws = {0, 0, 0, 0, 0, true};
        if (active) {
            const BubblyVertex v = bubbly_vertex<R>(jobs, bands, w, Pi, base + threadIdx.x, d, ng, cos_i, thick);
            i = v.i;
            tri = v.tri;
            const PathS<R> ps = rec_load(Pi.s + i);
            aux = ps.aux;
            pix = ps.pix;
            smp = ps.smp;
            const bool spec = (smp & kSpectral) != 0u;
            g = ps.g;
            const int depth = (int)(aux & 0xffu);
            const JobDev *jb = v.jb;
            const PathO<R> po = rec_load(Pi.o + i);
            x = V3<R>{po.x, po.y, po.z} + rec_load(w.hit + i).t * d;
            dnew = d;
            mo = (uint32_t)(v.mat * jb->ms + v.bd.l0);
            flags = (spec ? kRowSrc : 0u) | ((v.bd.l0 & 3) == 0 ? kRowAl : 0u) | (uint32_t)v.bd.nb << kRowNbShift |
                    (uint32_t)v.bd.l0 << 16;
            if (v.mode == kBtdfExact) {
                flags |= kRowExact;
                ws = {jb->seed, pix, smp & ~kSpectral, jb->job_word, (uint32_t)depth, true};
                R ue[4];
                walk_draw<R>(ws, 0, 0, ue);
                pol = ue[1] < R(0.5) ? 0 : 1;
                u0 = ue[0];
                sigma = R(v.sigma);
                n_ref = R(v.n_ref);
            } else {
                const uint4 rr = vertex_draws(jb->seed, jb->job_word, pix, smp & ~kSpectral, depth, 0);
                u0 = u01<R>(rr.x);
                dnew = lobe_dir<R>(d, w.bw[i], u01<R>(rr.y), u01<R>(rr.z));
                // a sample that points back through the entry side is
                // mirrored across the pane's plane: transmitted light leaves
                // on the far side
                const R dn_out = dot(dnew, ng);
                if (dn_out * dot(d, ng) < R(0)) dnew = dnew - (R(2) * dn_out) * ng;
            }
        }
        const RowTasks rt = row_tasks(active, nbm, s_map);
        // Row pass 1.  Exact: per wavelength with a weight, reflect where the
        // shared draw falls below the entry reflectance of the drawn
        // polarisation, else enter; the row holds +-b (b = 1 for a path
        // without per-wavelength factors).  Surrogate: the weights (already
        // times R + T) below the threshold are cleared, the others signed by
        // u0 < R / (R + T).
        bool anyR = false, anyT = false, enter = false;
        for (int b0 = 0; b0 < rt.n; b0 += rt.ng) {
            const int src = rt.src(b0, s_map);
            const uint32_t f = (uint32_t)__shfl((int)flags, src);
            const uint32_t si = (uint32_t)__shfl((int)i, src), smo = (uint32_t)__shfl((int)mo, src);
            const R sc = __shfl(cos_i, src), su = __shfl(u0, src), sg = __shfl(g, src);
            const int spol = __shfl(pol, src);
            const uint32_t sjob = (uint32_t)__shfl((int)(aux >> kAuxJobShift), src);
            const int nb = (int)((f >> kRowNbShift) & 0xffu), j = rt.j;
            bool lR = false, lT = false, lE = false;
            if (rt.busy(b0) && j < nb) {
                const JobDev *sj = &jobs[sjob];
                const bool al = (f & kRowAl) != 0u;
                R *__restrict__ brow = Pi.beta + aosoa(si, 0, nbm);
                Vec4<R> o4;
                if (f & kRowExact) {
                    Vec4<R> b4;
                    if (f & kRowSrc) b4 = row_load4(brow + j);
                    else b4.v[0] = b4.v[1] = b4.v[2] = b4.v[3] = R(1);
                    const Vec4<R> n4 = tab4((const R *)sj->n + smo, al, j, nb),
                                  k4 = tab4((const R *)sj->k + smo, al, j, nb);
#pragma unroll
                    for (int q = 0; q < 4; ++q) {
                        o4.v[q] = R(0);
                        if (j + q >= nb || b4.v[q] == R(0)) continue;
                        R Rs, Rp;
                        fresnel_sp<R>(sc, n4.v[q], k4.v[q], Rs, Rp);
                        if (su < (spol == 0 ? Rs : Rp)) o4.v[q] = -b4.v[q];
                        else {
                            o4.v[q] = b4.v[q];
                            lE = true;
                        }
                    }
                } else {
                    const Vec4<R> b4 = row_load4(brow + j), r4 = row_load4(w.bratio + aosoa(si, j, nbm));
                    const R thr = R(sj->beta_thr);
#pragma unroll
                    for (int q = 0; q < 4; ++q) {
                        o4.v[q] = R(0);
                        const R bn = b4.v[q];
                        if (j + q >= nb || bn == R(0) || sg * bn < thr) continue;
                        if (su < r4.v[q]) {
                            o4.v[q] = -bn;
                            lR = true;
                        } else {
                            o4.v[q] = bn;
                            lT = true;
                        }
                    }
                }
                row_store4(brow + j, o4);
            }
            const uint64_t bR = __ballot(lR), bT = __ballot(lT), bE = __ballot(lE);
            uint64_t mine;
            if (rt.mine(active, b0, mine)) {
                anyR = (bR & mine) != 0u;
                anyT = (bT & mine) != 0u;
                enter = (bE & mine) != 0u;
            }
        }
        // the walk of an exact vertex whose light enters the pane
        int wkind = 0;
        R wL = R(0);
        if (active && (flags & kRowExact) && enter) {
            const WalkOut<R> wo = bubbly_walk<R>(ws, cos_i, thick, sigma, n_ref, pol);
            wkind = wo.kind;
            wL = wo.L;
            if (wo.kind != 0) dnew = slab_to_world<R>(d, ng, wo.a);
        }
        // Row pass 2 (exact vertices): the reflected wavelengths keep their
        // weight, the entering ones take exp(-alpha L) if the walk left the
        // pane (zero if it was absorbed); then the energy threshold.
        for (int b0 = 0; b0 < rt.n; b0 += rt.ng) {
            const int src = rt.src(b0, s_map);
            const uint32_t f = (uint32_t)__shfl((int)flags, src);
            const uint32_t si = (uint32_t)__shfl((int)i, src), smo = (uint32_t)__shfl((int)mo, src);
            const R sg = __shfl(g, src), sL = __shfl(wL, src);
            const int sk = __shfl(wkind, src);
            const uint32_t sjob = (uint32_t)__shfl((int)(aux >> kAuxJobShift), src);
            const int nb = (int)((f >> kRowNbShift) & 0xffu), j = rt.j;
            bool lR = false, lT = false;
            if (rt.busy(b0) && j < nb && (f & kRowExact)) {
                const JobDev *sj = &jobs[sjob];
                const bool al = (f & kRowAl) != 0u;
                R *__restrict__ brow = Pi.beta + aosoa(si, 0, nbm);
                const Vec4<R> b4 = row_load4(brow + j);
                const Vec4<R> l4 = tab4((const R *)sj->lam + (f >> 16), al, j, nb),
                              k4 = tab4((const R *)sj->k + smo, al, j, nb),
                              t4 = tab4((const R *)sj->tint + smo, al, j, nb);
                const R thr = R(sj->beta_thr);
                Vec4<R> o4;
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    o4.v[q] = R(0);
                    const R b = b4.v[q];
                    if (j + q >= nb || b == R(0)) continue;
                    const bool refl = b < R(0);
                    R bn = R(0);
                    if (refl) {
                        bn = -b;
                    } else if (sk != 0) {
                        const R alpha = R(12.566370614359172) * k4.v[q] / (l4.v[q] * R(1e-6)) + t4.v[q];
                        bn = b * exp(-alpha * sL);
                    }
                    if (sg * bn < thr) bn = R(0);
                    if (bn == R(0)) continue;
                    if (refl) {
                        o4.v[q] = -bn;
                        lR = true;
                    } else {
                        o4.v[q] = bn;
                        lT = true;
                    }
                }
                row_store4(brow + j, o4);
            }
            const uint64_t bR = __ballot(lR), bT = __ballot(lT);
            uint64_t mine;
            if (rt.mine(active && (flags & kRowExact), b0, mine)) {
                anyR = (bR & mine) != 0u;
                anyT = (bT & mine) != 0u;
            }
        }
        bool keep = anyR || anyT, fork = anyR && anyT;
        const V3<R> drefl = d - (R(2) * dot(d, ng)) * ng;
        if (anyR && !anyT) dnew = drefl;
        n_fork += fork ? 1u : 0u;
        uint32_t om, of;
        emit_paths<R>(w, Po, cur, keep, fork, x, dnew, drefl, pix, smp, aux, tri, g, om, of, s_cnt, s_base);
        // the rows of the outputs: the kept path takes the transmitted
        // wavelengths (all of them without a fork), the forked path the
        // reflected ones
        const uint32_t ef = flags | (keep ? kRowKeep : 0u) | (fork ? kRowFork : 0u);
        for (int b0 = 0; b0 < rt.n; b0 += rt.ng) {
            const int src = rt.src(b0, s_map);
            const uint32_t f = (uint32_t)__shfl((int)ef, src);
            const uint32_t si = (uint32_t)__shfl((int)i, src), so = (uint32_t)__shfl((int)om, src),
                           sf = (uint32_t)__shfl((int)of, src);
            const int nb = (int)((f >> kRowNbShift) & 0xffu), j = rt.j;
            if (!rt.busy(b0) || j >= nb || !(f & kRowKeep)) continue;
            const bool fk = (f & kRowFork) != 0u;
            const Vec4<R> b = row_load4(Pi.beta + aosoa(si, j, nbm));
            Vec4<R> k4, f4;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const bool refl = signbit(b.v[q]);
                const R a = fabs(b.v[q]);
                k4.v[q] = (fk && refl) ? R(0) : a;
                f4.v[q] = refl ? a : R(0);
            }
            row_store4(Po.beta + aosoa(so, j, nbm), k4);
            if (fk) row_store4(Po.beta + aosoa(sf, j, nbm), f4);
        }
    }
    for (int off = 32; off > 0; off >>= 1) n_fork += __shfl_xor(n_fork, off);
    if (lane == 0 && n_fork) atomicAdd(&w.cnt->forks, (unsigned long long)n_fork);
}

// ---------------------------------------------------------------------------
// Shadow records: any-hit walk toward the sun.  socc = -1 when an opaque
// triangle is in the way, else the number of panes crossed, kept for the
// transmittance pass.  A walk that crosses more than kMaxGlass panes sets
// bit 1 of the overflow word and the render reports it.
// ---------------------------------------------------------------------------
template <class R, bool kOne>
__global__ void __launch_bounds__(kBlock) k_shadow_trace(const JobDev *__restrict__ jobs, const BandDev *__restrict__ bands, Work<R> w,
                                                         int lds_job)
{
    if (lds_job < -1) lds_job = w.cnt->lds_job;
    __shared__ float4 s_nodes[8 * kLdsNodes];
    __shared__ int32_t s_stack[kLdsStack * kBlock];
    const uint32_t count = min(w.cnt->scount, w.cap);
    if (blockIdx.x == 0 && threadIdx.x == 0) w.cnt->shadow += count;
    // a scene whose shadow rays use the sun grid needs no BVH prefix
    const int n_lds = lds_job >= 0 && !jobs[lds_job].sc.g_use ? stage_nodes(s_nodes, jobs[lds_job].sc) : 0;
    Stack st = make_stack(s_stack, w.gstack_sh);
    WaveFeed feed{0, 0, false, 0};
    Ray<R> ry;
    GridRange<R> gr{0, 0, R(0)};
    int64_t item = -1;
    int job = 0, ng = 0;
    bool occ = false, over = false, grid = false, away = false;
    R teps = R(0);
    uint32_t n_nodes = 0, n_tests = 0;
    for (;;) {
        const int64_t got = feed.next(item < 0, count);
        if (got >= 0) {
            item = got;
            const uint32_t s = (uint32_t)got;
            job = kOne ? 0 : (int)(w.saux[s] >> kAuxJobShift);
            const SceneDev &sc = jobs[job].sc;
            grid = sc.g_use != 0;
            const V3<R> o = {w.sx[s], w.sy[s], w.sz[s]}, d = {R(sc.sun[0]), R(sc.sun[1]), R(sc.sun[2])};
            if (grid) {   // the candidate walk needs no slab setup, only the triangle test's shear
                ry.o = o;
                ry.d = d;
                if constexpr (sizeof(R) == 4) ry.sh = make_shear(o, d);
                gr = grid_range(sc, o);
            } else {
                set_dir(ry, o, d);
            }
            ry.skip = w.sskip[s];
            ry.cur = !grid && sc.n_nodes > 0 ? 0 : kDone;
            teps = teps_of<R>(sc);
            ng = 0;
            // a record whose sun term is zero (a surface facing away from the
            // sun, kept for the caustic gather) needs no walk
            away = jobs[job].caustic && w.scs[s] == R(0);
            occ = false;
            over = false;
            st.sp = 0;
        }
        if (!__ballot(item >= 0)) {
            if (feed.done) break;
            continue;
        }
        if (item >= 0) {
            const uint32_t rec = (uint32_t)item;
            auto on_glass = [&](int leaf, int mat, R u, R v) {
                if (ng == kMaxGlass) {
                    over = true;
                    return;
                }
                const SceneDev &scj = jobs[job].sc;
                int m;
                R dd;
                pane_at<R>(scj, leaf, mat, u, v, m, dd);
                w.sg_leaf[(size_t)rec * kMaxGlass + ng] = leaf;
                w.sg_d[(size_t)rec * kMaxGlass + ng] = dd;
                w.sg_m[(size_t)rec * kMaxGlass + ng] = m;
                ++ng;
            };
            bool fin;
            if (away) {
                fin = true;
                occ = true;
            } else if (grid)
                fin = grid_step(jobs[job].sc, ry, gr, occ, teps, on_glass, n_nodes, n_tests);
            else
                fin = ry.cur == kDone || shadow_step<true>(jobs[job].sc, s_nodes, job == lds_job ? n_lds : 0, st, ry,
                                                           occ, teps, on_glass, n_nodes, n_tests);
            if (fin) {
                // an occluded walk needs no pane list, whatever the visiting order found first
                if (over && !occ) atomicOr(&w.cnt->overflow, 2u);
                w.socc[rec] = occ ? -1 : ng;
                item = -1;
            }
        }
    }
    if (n_nodes) {
        atomicAdd(&w.cnt->nodes[1], (unsigned long long)n_nodes);
        atomicAdd(&w.cnt->tris[1], (unsigned long long)n_tests);
    }
}

// Per wavelength: the record's contribution times the slab transmittance of
// each pane crossed (at the sun angle, thickness at the crossing) -- or, for
// the sky record of an escaped path, its weight times the sky radiance --
// added to the FP64 accumulator row of its pixel.
//
// The accumulator's FP64 atomic adds are performed on the memory side, one
// request per lane address, so the pass is arranged for few, contiguous
// atomics.  Wave w takes the nominal groups w, w + W, w + 2W, ... of
// kAccGroup records (W waves; interleaved because occlusion and pane counts
// vary along the record buffer), each moved to start and end where the
// pixel changes.  Batches of up to 64 unoccluded records go through two
// phases: lanes over records compute each record's setup (pane cosines,
// thicknesses, materials) into LDS; then lanes over wavelengths walk the
// batch's records in order, summing a pixel's records in registers (also
// across batches) and adding the row with one atomic instruction per 64
// consecutive wavelengths when the pixel changes.
constexpr uint32_t kAccGroup = 64;   // nominal records per group of the accumulation pass
constexpr int kAccPanes = 2;         // panes per record held in LDS (more are read again from the record)

template <class R>
struct AccRec {
    uint64_t key;        // accumulator row (its wavelength l0 included)
    R scs;               // scalar factor
    uint32_t rec;        // record slot (per-wavelength factors, further panes)
    int32_t job, l0, nb, ng;
    int32_t flags;       // bit 0: spectral factors, bit 1: sky record
    R c[kAccPanes], d[kAccPanes], sig[kAccPanes];
    int32_t m[kAccPanes];
};

template <class R>
__device__ __forceinline__ void pane_geometry(const JobDev *jb, const Work<R> &w, uint32_t rec, int g, R &c, R &d,
                                              int &m, R &sig)
{
    const V3<R> sun = {R(jb->sc.sun[0]), R(jb->sc.sun[1]), R(jb->sc.sun[2])};
    const int leaf = w.sg_leaf[(size_t)rec * kMaxGlass + g];
    const TriDev tr = load_tri(jb->sc.tris, leaf);
    c = fabs(dot(sun, tri_normal<R>(tr)));
    d = w.sg_d[(size_t)rec * kMaxGlass + g];
    m = w.sg_m[(size_t)rec * kMaxGlass + g];
    // toward the delta sun a bubbly pane passes its unscattered light: the
    // bubbles' extinction adds to the absorption
    sig = R(gld(jb->sc.mat_bub + 4 * m));
}

// FP32: six waves per SIMD (measured best; eight spill too much)
template <class R, bool kOne>
__global__ void __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(sizeof(R) == 4 ? 6 : 1))) k_shadow_accum(const JobDev *__restrict__ jobs,
                                                         const BandDev *__restrict__ bands, Work<R> w)
{
    __shared__ uint32_t s_buf[kBlock / 64][128];
    __shared__ AccRec<R> s_rec[kBlock / 64][64];
    // sun records [0, ns), then the sky records of escaped paths stored from
    // the back of the buffer (one record per path, so the ranges are disjoint)
    const uint32_t ns = min(w.cnt->scount, w.cap);
    const uint32_t nk = min(w.cnt->kcount, w.cap - ns);
    const uint32_t count = ns + nk;
    const int nbm = w.nbmax;
    const uint32_t lane = lane_id();
    const uint64_t lt = (1ull << lane) - 1ull;
    const uint32_t wv = threadIdx.x >> 6;
    uint32_t *buf = s_buf[wv];
    AccRec<R> *rb = s_rec[wv];
    const uint32_t nwaves = (gridDim.x * blockDim.x) >> 6;
    auto rec_of = [&](uint32_t i) { return i < ns ? i : w.cap - 1u - (i - ns); };
    // records of one accumulator row (job, band, pixel) share this key
    auto key_at = [&](uint32_t i) {
        const uint32_t r = rec_of(i);
        return ((uint64_t)(w.saux[r] >> kAuxBandShift) << 32) | (w.spix[r] & ~kSpectral);
    };
    // first index >= x that starts a run of equal keys (all lanes together)
    auto run_start_at = [&](uint32_t x) -> uint32_t {
        if (x == 0 || x >= count) return min(x, count);
        const uint64_t kp = key_at(x - 1);
        for (uint32_t y = x; y < count; y += 64) {
            const uint32_t i = y + lane;
            const uint64_t m = __ballot(i >= count || key_at(i) != kp);
            if (m) return min(count, y + (uint32_t)__ffsll((unsigned long long)m) - 1u);
        }
        return count;
    };
    // the row being summed (wave-uniform) and its sums at wavelengths lane and lane + 64
    uint64_t row = ~0ull;
    int row_nb = 0;
    // table values cached per lane across records (see phase 2)
    uint32_t c_skey = ~0u, c_mkey = ~0u;
    R c_E[2] = {R(0), R(0)}, c_lam[2] = {R(0), R(0)}, c_n[2] = {R(0), R(0)}, c_k[2] = {R(0), R(0)}, c_t[2] = {R(0), R(0)};
    double s0 = 0.0, s1 = 0.0;
    auto flush = [&]() {
        if (row != ~0ull) {
            if ((int)lane < row_nb && s0 != 0.0) unsafeAtomicAdd(w.acc + row + lane, s0);
            if ((int)lane + 64 < row_nb && s1 != 0.0) unsafeAtomicAdd(w.acc + row + lane + 64, s1);
        }
        s0 = s1 = 0.0;
    };
    uint32_t g = (blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    uint32_t base = 0, gb = 0, nbuf = 0;
    bool groups_left = true;
    for (;;) {
        while (nbuf < 64 && groups_left) {
            if (base >= gb) {   // next group of this wave
                if ((uint64_t)g * kAccGroup >= count) {
                    groups_left = false;
                    break;
                }
                base = run_start_at(g * kAccGroup);
                gb = run_start_at((uint32_t)min<uint64_t>((uint64_t)(g + 1) * kAccGroup, count));
                g += nwaves;
                continue;
            }
            const uint32_t i = base + lane;
            const bool ok = i < gb && (i >= ns || w.socc[i] >= 0);
            const uint64_t m = __ballot(ok);
            if (ok) buf[nbuf + (uint32_t)__popcll(m & lt)] = rec_of(i);
            nbuf += (uint32_t)__popcll(m);
            base = min(gb, base + 64u);
        }
        __builtin_amdgcn_wave_barrier();
        if (nbuf == 0) break;
        const uint32_t take = min(nbuf, 64u);
        // phase 1, lanes over records: each record's setup
        if (lane < take) {
            const uint32_t rec = buf[lane];
            AccRec<R> a;
            const bool sky = rec >= ns;
            const uint32_t aux = w.saux[rec];
            a.job = kOne ? 0 : (int)(aux >> kAuxJobShift);
            const JobDev *jb = &jobs[a.job];
            const BandDev bd = bands[(aux >> kAuxBandShift) & ((1u << kAuxBandBits) - 1u)];
            const uint32_t sp = w.spix[rec];
            a.rec = rec;
            a.l0 = bd.l0;
            a.nb = bd.nb;
            a.ng = sky ? 0 : w.socc[rec];
            a.flags = ((sp & kSpectral) ? 1 : 0) | (sky ? 2 : 0);
            a.scs = w.scs[rec];
            a.key = jb->acc_off + (uint64_t)(sp & ~kSpectral) * jb->nl + bd.l0;
#pragma unroll
            for (int q = 0; q < kAccPanes; ++q) {
                if (q < a.ng) {
                    pane_geometry(jb, w, rec, q, a.c[q], a.d[q], a.m[q], a.sig[q]);
                } else {
                    a.c[q] = a.d[q] = a.sig[q] = R(0);
                    a.m[q] = 0;
                }
            }
            rb[lane] = a;
        }
        __builtin_amdgcn_wave_barrier();
        // phase 2, lanes over wavelengths: the batch's records in order
        for (uint32_t r = 0; r < take; ++r) {
            const AccRec<R> a = rb[r];
            if (a.key != row) {
                flush();
                row = a.key;
                row_nb = a.nb;
            }
            const JobDev *jb = &jobs[kOne ? 0 : a.job];
            const R *tn = (const R *)jb->n, *tk = (const R *)jb->k, *tt = (const R *)jb->tint;
            const int ms = jb->ms;
            // this lane's table values (wavelengths lane and lane + 64), reloaded
            // only when the band, the light or the first pane's material changes
            const uint32_t skey = (uint32_t)a.job << 20 | (uint32_t)a.l0 << 1 | (uint32_t)((a.flags >> 1) & 1);
            if (skey != c_skey) {
                c_skey = skey;
                const R *spectrum = (const R *)((a.flags & 2) ? jb->Lsky : jb->E);
                const R *lam = (const R *)jb->lam;
#pragma unroll
                for (int h = 0; h < 2; ++h) {
                    const int l = a.l0 + min((int)lane + 64 * h, a.nb - 1);
                    c_E[h] = gld(spectrum + l);
                    c_lam[h] = gld(lam + l);
                }
                c_mkey = ~0u;
            }
            if (a.ng > 0) {
                const uint32_t mkey = (uint32_t)a.m[0];
                if (mkey != c_mkey) {
                    c_mkey = mkey;
#pragma unroll
                    for (int h = 0; h < 2; ++h) {
                        const size_t mo = (size_t)a.m[0] * ms + a.l0 + min((int)lane + 64 * h, a.nb - 1);
                        c_n[h] = gld(tn + mo);
                        c_k[h] = gld(tk + mo);
                        c_t[h] = gld(tt + mo);
                    }
                }
            }
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const int j = (int)lane + 64 * h;
                if (j >= a.nb) continue;
                const int l = a.l0 + j;
                R T = a.scs * c_E[h];
                if (a.flags & 1) T *= w.contrib[aosoa(a.rec, j, nbm)];
                const R lamv = c_lam[h];
#pragma unroll
                for (int q = 0; q < kAccPanes; ++q) {
                    if (q < a.ng) {
                        R Rr, Tt;
                        if (a.m[q] == a.m[0]) {
                            slab_RT<R>(a.c[q], lamv, a.d[q], c_n[h], c_k[h], c_t[h] + a.sig[q], Rr, Tt);
                        } else {
                            const size_t mo = (size_t)a.m[q] * ms + l;
                            slab_RT<R>(a.c[q], lamv, a.d[q], gld(tn + mo), gld(tk + mo), gld(tt + mo) + a.sig[q], Rr, Tt);
                        }
                        T *= Tt;
                    }
                }
                for (int q = kAccPanes; q < a.ng; ++q) {   // rare: further panes, set up again here
                    R c, d, sig;
                    int m;
                    pane_geometry(jb, w, a.rec, q, c, d, m, sig);
                    const size_t mo = (size_t)m * ms + l;
                    R Rr, Tt;
                    slab_RT<R>(c, lamv, d, gld(tn + mo), gld(tk + mo), gld(tt + mo) + sig, Rr, Tt);
                    T *= Tt;
                }
                if (h == 0) s0 += (double)T;
                else s1 += (double)T;
            }
        }
        // keep the records not processed yet at the front of the buffer
        const uint32_t rem = nbuf - take;
        const uint32_t nxt = lane < rem ? buf[take + lane] : 0u;
        __builtin_amdgcn_wave_barrier();
        if (lane < rem) buf[lane] = nxt;
        __builtin_amdgcn_wave_barrier();
        nbuf = rem;
    }
    flush();
}

// ---------------------------------------------------------------------------
// Event signatures (debug): per spectral pixel, the sum modulo 2^64 of a hash
// of every event that decides what its paths contribute -- each closest hit
// (vertex, sample, triangle or none) and each shadow-ray result (vertex,
// occluded or the set of panes crossed) -- counted for the wavelengths whose
// weight is nonzero.  Renders whose paths take the same decisions give equal
// sums, so a pixel whose sum differs from a reference's holds a path that
// decided differently (a flip).  The hash is the output function of
// SplitMix64 (Steele, Lea and Flood, OOPSLA 2014) on a packed event word:
// kind << 56 | vertex << 48 | low 48 bits (sample << 32 | triangle + 1 for a
// hit; 0xFFFF when occluded, else the pane count, for a shadow ray, plus the
// hashes of kind 3 with each pane's triangle).
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint64_t ev_mix(uint64_t z)
{
    z += 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

template <class R>
__global__ void __launch_bounds__(kBlock) k_sig_hits(const JobDev *__restrict__ jobs, const BandDev *__restrict__ bands,
                                                     Work<R> w, int cur)
{
    const uint32_t count = min(w.cnt->count[cur], w.cap);
    const Pool<R> P = w.p[cur];
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < count; i += gridDim.x * blockDim.x) {
        const PathS<R> ps = rec_load(P.s + i);
        if (ps.g == R(0)) continue;
        const HitRec<R> hr = rec_load(w.hit + i);
        const JobDev &jb = jobs[ps.aux >> kAuxJobShift];
        const BandDev bd = bands[(ps.aux >> kAuxBandShift) & ((1u << kAuxBandBits) - 1u)];
        const int32_t caller = hr.tri >= 0 ? __float_as_int(load_tri(jb.sc.tris, hr.tri).a.w) : -1;
        const uint64_t key = ev_mix(1ull << 56 | (uint64_t)(ps.aux & 0xffu) << 48 |
                                    (uint64_t)(ps.smp & ~kSpectral) << 32 | (uint32_t)(caller + 1));
        unsigned long long *row = w.sig + jb.acc_off + (uint64_t)ps.pix * jb.nl + bd.l0;
        const bool spec = (ps.smp & kSpectral) != 0u;
        for (int j = 0; j < bd.nb; ++j)
            if (!spec || P.beta[aosoa(i, j, w.nbmax)] != R(0)) atomicAdd(row + j, (unsigned long long)key);
    }
}

template <class R>
__global__ void __launch_bounds__(kBlock) k_sig_shadow(const JobDev *__restrict__ jobs, const BandDev *__restrict__ bands,
                                                       Work<R> w)
{
    const uint32_t ns = min(w.cnt->scount, w.cap);
    for (uint32_t r = blockIdx.x * blockDim.x + threadIdx.x; r < ns; r += gridDim.x * blockDim.x) {
        if (w.scs[r] == R(0)) continue;
        const uint32_t sp = w.spix[r], aux = w.saux[r];
        const JobDev &jb = jobs[aux >> kAuxJobShift];
        const BandDev bd = bands[(aux >> kAuxBandShift) & ((1u << kAuxBandBits) - 1u)];
        const int occ = w.socc[r];
        uint64_t key = ev_mix(2ull << 56 | (uint64_t)(aux & 0xffu) << 48 | (occ < 0 ? 0xFFFFull : (uint64_t)occ));
        for (int q = 0; q < min(occ, kMaxGlass); ++q) {
            const int leaf = w.sg_leaf[(size_t)r * kMaxGlass + q];
            key += ev_mix(3ull << 56 | (uint32_t)__float_as_int(load_tri(jb.sc.tris, leaf).a.w));
        }
        unsigned long long *row = w.sig + jb.acc_off + (uint64_t)(sp & ~kSpectral) * jb.nl + bd.l0;
        const bool spec = (sp & kSpectral) != 0u;
        for (int j = 0; j < bd.nb; ++j)
            if (!spec || w.contrib[aosoa(r, j, w.nbmax)] != R(0)) atomicAdd(row + j, (unsigned long long)key);
    }
}

// ---------------------------------------------------------------------------
// Accumulator -> mean spectral radiance (float) and XYZ (FP64):
// XYZ = sum_i w_i L(lambda_i) cmf_i with trapezoid weights.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(kBlock) k_finalize(const double *acc, int64_t npix, int nl, int spp,
                                                     const double *wts, const double *cmf, float *spec,
                                                     double *xyz)
{
    // one wave per pixel, lanes over wavelengths: the row is read and the
    // spectrum written contiguously; the XYZ sums are reduced across the wave
    const uint32_t lane = lane_id();
    const int64_t nw = ((int64_t)gridDim.x * blockDim.x) >> 6;
    for (int64_t p = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) >> 6; p < npix; p += nw) {
        double X = 0.0, Y = 0.0, Z = 0.0;
        const double *a = acc + p * nl;
        for (int l = (int)lane; l < nl; l += 64) {
            const double v = a[l] / spp;
            if (spec) spec[p * nl + l] = (float)v;
            const double wv = wts[l] * v;
            X += wv * cmf[3 * l];
            Y += wv * cmf[3 * l + 1];
            Z += wv * cmf[3 * l + 2];
        }
        for (int off = 32; off > 0; off >>= 1) {
            X += __shfl_xor(X, off);
            Y += __shfl_xor(Y, off);
            Z += __shfl_xor(Z, off);
        }
        if (xyz && lane == 0) {
            xyz[3 * p] = X;
            xyz[3 * p + 1] = Y;
            xyz[3 * p + 2] = Z;
        }
    }
}

__global__ void k_zero_f64(double *a, int64_t n)
{
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += stride) a[i] = 0.0;
}

__global__ void k_advance_cursor(Counters *c, uint32_t chunk)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) c->r0 += chunk;
}

// The record queues of a bounce (shadow, sky, glass and bubbly vertices)
// emptied for the next one, after their last reader: the closest-hit pass of
// the next bounce may run meanwhile, so it cannot clear them itself.
__global__ void k_reset_records(Counters *c)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) c->scount = c->kcount = c->gcount = c->bcount = 0;
}

__global__ void k_zero_counters(Counters *c)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        c->r0 = 0;
        c->lds_job = 0;
        c->count[0] = c->count[1] = 0;
        c->scount = c->kcount = 0;
        c->overflow = 0;
        c->gcount = c->bcount = 0;
        c->closest = c->shadow = c->forks = c->bubbly = 0;
        c->spec_paths = c->spec_records = 0;
        c->glass[0] = c->glass[1] = 0;
        c->nodes[0] = c->nodes[1] = c->tris[0] = c->tris[1] = 0;
        c->interface_rays = 0;
        c->ddn[0] = c->ddn[1] = c->ddn[2] = 0;
        c->phcount = 0;
    }
}

// Linear interpolation of a table (tab_x[n_tab], tab_y[n_tab]) at xs[nl],
// held constant beyond the ends; `rows` tables, written as rows of `stride`
// (>= nl) values whose padding is set to zero.
template <class R>
__global__ void k_resample(const float *tab_x, int n_tab, const float *tab_y, int rows, const float *xs, int nl,
                           int stride, R *out)
{
    const int total = rows * stride;
    for (int id = blockIdx.x * blockDim.x + threadIdx.x; id < total; id += gridDim.x * blockDim.x) {
        const int r = id / stride, l = id % stride;
        if (l >= nl) {
            out[id] = R(0);
            continue;
        }
        const float *y = tab_y + (size_t)r * n_tab;
        const double x = xs[l];
        double v;
        if (n_tab == 1 || x <= tab_x[0]) {
            v = y[0];
        } else if (x >= tab_x[n_tab - 1]) {
            v = y[n_tab - 1];
        } else {
            int i = 0;
            while ((double)tab_x[i + 1] < x) ++i;
            const double wgt = (x - tab_x[i]) / ((double)tab_x[i + 1] - tab_x[i]);
            v = (1.0 - wgt) * y[i] + wgt * y[i + 1];
        }
        out[id] = (R)v;
    }
}

// ---------------------------------------------------------------------------
// Test hooks: batch slab optics, closest hit and sun transmittance.
// ---------------------------------------------------------------------------
__global__ void k_slab_eval(int64_t m, const float *c, const float *lam, const float *d, const float *n,
                            const float *k, const float *tint, float *R, float *T)
{
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < m; i += stride) {
        float r, t;
        slab_RT<float>(c[i], lam[i], d[i], n[i], k[i], tint ? tint[i] : 0.0f, r, t);
        R[i] = r;
        T[i] = t;
    }
}

__global__ void __launch_bounds__(kBlock) k_debug_intersect(SceneDev sc, uint32_t m, const float *o, const float *d,
                                                            const int32_t *skip, const int32_t *orig_to_leaf,
                                                            float *t, int32_t *tri, float *uv,
                                                            int32_t *gstack)
{
    __shared__ float4 s_nodes[8 * kLdsNodes];
    __shared__ int32_t s_stack[kLdsStack * kBlock];
    const int n_lds = stage_nodes(s_nodes, sc);
    Stack st = make_stack(s_stack, gstack);
    WaveFeed feed{0, 0, false, 0};
    Ray<float> ry;
    Closest<float> h;
    int64_t item = -1;
    uint32_t nn = 0, nt = 0;
    for (;;) {
        const int64_t got = feed.next(item < 0, m);
        if (got >= 0) {
            item = got;
            set_dir(ry, V3<float>{o[3 * got], o[3 * got + 1], o[3 * got + 2]},
                    V3<float>{d[3 * got], d[3 * got + 1], d[3 * got + 2]});
            ry.skip = (skip && skip[got] >= 0 && skip[got] < sc.nt) ? orig_to_leaf[skip[got]] : -1;
            ry.cur = sc.n_nodes > 0 ? 0 : kDone;
            h.tb = INFINITY; h.ub = h.vb = 0.0f; h.trib = -1; h.orig_b = INT_MAX;
            st.sp = 0;
        }
        if (!__ballot(item >= 0)) {
            if (feed.done) break;
            continue;
        }
        if (item >= 0) {
            const bool fin = ry.cur == kDone || closest_step<false>(sc, s_nodes, n_lds, st, ry, h, sc.teps_f, nn, nt);
            if (fin) {
                t[item] = h.tb;
                tri[item] = h.trib >= 0 ? __float_as_int(sc.tris[h.trib].a.w) : -1;
                uv[2 * item] = h.ub;
                uv[2 * item + 1] = h.vb;
                item = -1;
            }
        }
    }
}

__global__ void __launch_bounds__(kBlock) k_debug_shadow(SceneDev sc, uint32_t m, const float *o, const int32_t *skip,
                                                         const int32_t *orig_to_leaf, float lambda_nm,
                                                         const float *n_at, const float *k_at, const float *t_at,
                                                         float *T, int32_t *gstack)
{
    __shared__ float4 s_nodes[8 * kLdsNodes];
    __shared__ int32_t s_stack[kLdsStack * kBlock];
    const int n_lds = stage_nodes(s_nodes, sc);
    Stack st = make_stack(s_stack, gstack);
    WaveFeed feed{0, 0, false, 0};
    Ray<float> ry;
    int64_t item = -1;
    bool occ = false;
    float prod = 1.0f;
    GridRange<float> gr{0, 0, 0.0f};
    uint32_t nn = 0, nt = 0;
    const V3<float> sun = {sc.sun[0], sc.sun[1], sc.sun[2]};
    for (;;) {
        const int64_t got = feed.next(item < 0, m);
        if (got >= 0) {
            item = got;
            set_dir(ry, V3<float>{o[3 * got], o[3 * got + 1], o[3 * got + 2]}, sun);
            ry.skip = (skip && skip[got] >= 0 && skip[got] < sc.nt) ? orig_to_leaf[skip[got]] : -1;
            if (sc.g_use) gr = grid_range(sc, ry.o);
            ry.cur = !sc.g_use && sc.n_nodes > 0 ? 0 : kDone;
            occ = false;
            prod = 1.0f;
            st.sp = 0;
        }
        if (!__ballot(item >= 0)) {
            if (feed.done) break;
            continue;
        }
        if (item >= 0) {
            auto on_glass = [&](int leaf, int mat, float u, float v) {
                const TriDev tr = load_tri(sc.tris, leaf);
                int mt;
                float dm;
                pane_at<float>(sc, leaf, mat, u, v, mt, dm);
                float Rr, Tt;
                slab_RT<float>(fabsf(dot(sun, tri_normal<float>(tr))), lambda_nm, dm, n_at[mt], k_at[mt],
                               t_at[mt] + (float)gld(sc.mat_bub + 4 * mt), Rr, Tt);
                prod *= Tt;
            };
            // the walk of the render: the sun grid where the scene has one (test
            // origins lie in the scene's bounds, as render origins do), else the BVH
            const bool fin = sc.g_use ? grid_step(sc, ry, gr, occ, sc.teps_f, on_glass, nn, nt)
                                      : (ry.cur == kDone ||
                                         shadow_step<false>(sc, s_nodes, n_lds, st, ry, occ, sc.teps_f, on_glass, nn, nt));
            if (fin) {
                T[item] = occ ? 0.0f : prod;
                item = -1;
            }
        }
    }
}

// ---------------------------------------------------------------------------
// Host launchers
// ---------------------------------------------------------------------------
template <class R>
void launch_generate(const JobDev *jobs, const BandDev *bands, const ItemDev *items, int n_items, const Work<R> &w,
                     uint64_t total, uint32_t chunk, int grid, hipStream_t s)
{
    hipLaunchKernelGGL(k_generate<R>, dim3(grid), dim3(kBlock), 0, s, jobs, bands, items, n_items, w, total, chunk);
}
template <class R>
void launch_trace(const JobDev *jobs, const Work<R> &w, int cur, int lds_job, bool surface, bool one_job, int grid,
                  hipStream_t s)
{
    const dim3 g(grid), b(kTraceBlock);
    if (one_job) {
        if (surface) hipLaunchKernelGGL((k_trace<R, true, true>), g, b, 0, s, jobs, w, cur, lds_job);
        else hipLaunchKernelGGL((k_trace<R, false, true>), g, b, 0, s, jobs, w, cur, lds_job);
    } else {
        if (surface) hipLaunchKernelGGL((k_trace<R, true, false>), g, b, 0, s, jobs, w, cur, lds_job);
        else hipLaunchKernelGGL((k_trace<R, false, false>), g, b, 0, s, jobs, w, cur, lds_job);
    }
}
template <class R>
void launch_photon_pass(const JobDev *jobs, const PhotonWork<R> &pw, int grid_trace, int num_cu, hipStream_t s)
{
    hipLaunchKernelGGL(k_ph_clear<R>, dim3(4 * num_cu), dim3(kBlock), 0, s, pw);
    hipLaunchKernelGGL(k_photon<R>, dim3(grid_trace), dim3(kTraceBlock), 0, s, jobs, pw);
    hipLaunchKernelGGL(k_ph_count<R>, dim3(4 * num_cu), dim3(kBlock), 0, s, pw);
    // the buckets' counts and a final 0 (start[buckets] = total); at most
    // 2^23 + 1 values, so the block totals (pw.nblk <= 4096) fit one block
    const uint32_t nv = pw.mask + 2u;
    hipLaunchKernelGGL(k_scan_blocks, dim3(pw.nblk), dim3(kScanBlock), 0, s, pw.start, nv, pw.part);
    hipLaunchKernelGGL(k_scan_blocks, dim3(1), dim3(kScanBlock), 0, s, pw.part, pw.nblk, (uint32_t *)nullptr);
    hipLaunchKernelGGL(k_scan_add, dim3(pw.nblk), dim3(kScanBlock), 0, s, pw.start, nv, (const uint32_t *)pw.part);
    hipLaunchKernelGGL(k_ph_place<R>, dim3(4 * num_cu), dim3(kBlock), 0, s, pw);
}
template <class R>
void launch_caustic(const JobDev *jobs, const BandDev *bands, const Work<R> &w, const PhotonWork<R> &pw, int grid,
                    hipStream_t s)
{
    hipLaunchKernelGGL(k_caustic<R>, dim3(grid), dim3(kBlock), 0, s, jobs, bands, w, pw);
}
template <class R>
void launch_dd_trace(const JobDev *jobs, const Work<R> &w, int cur, bool surface, int sweeps, bool march, int grid,
                     hipStream_t s)
{
    const dim3 g(grid), b(kTraceBlock);
    if (march) {
        if (surface) hipLaunchKernelGGL((k_dd_sweep<R, true, true, true>), g, b, 0, s, jobs, w, cur, 0, 1);
        else hipLaunchKernelGGL((k_dd_sweep<R, false, true, true>), g, b, 0, s, jobs, w, cur, 0, 1);
        return;
    }
    for (int k = 0; k < sweeps; ++k) {
        const int last = k == sweeps - 1;
        if (k == 0) {
            if (surface) hipLaunchKernelGGL((k_dd_sweep<R, true, true, false>), g, b, 0, s, jobs, w, cur, k, last);
            else hipLaunchKernelGGL((k_dd_sweep<R, false, true, false>), g, b, 0, s, jobs, w, cur, k, last);
        } else {
            if (surface) hipLaunchKernelGGL((k_dd_sweep<R, true, false, false>), g, b, 0, s, jobs, w, cur, k, last);
            else hipLaunchKernelGGL((k_dd_sweep<R, false, false, false>), g, b, 0, s, jobs, w, cur, k, last);
        }
    }
}
template <class R>
void launch_shade(const JobDev *jobs, const BandDev *bands, const Work<R> &w, int cur, bool one_job, int grid,
                  hipStream_t s)
{
    if (one_job) hipLaunchKernelGGL((k_shade<R, true>), dim3(grid), dim3(kShadeBlock), 0, s, jobs, bands, w, cur);
    else hipLaunchKernelGGL((k_shade<R, false>), dim3(grid), dim3(kShadeBlock), 0, s, jobs, bands, w, cur);
}
template <class R>
void launch_shade_glass(const JobDev *jobs, const BandDev *bands, const Work<R> &w, int cur, bool one_job, int grid,
                        hipStream_t s)
{
    if (one_job) hipLaunchKernelGGL((k_shade_glass<R, true>), dim3(grid), dim3(kBlock), 0, s, jobs, bands, w, cur);
    else hipLaunchKernelGGL((k_shade_glass<R, false>), dim3(grid), dim3(kBlock), 0, s, jobs, bands, w, cur);
}
template <class R>
void launch_bubbly_eval(const JobDev *jobs, const BandDev *bands, const Work<R> &w, int cur, const float *params,
                        const float *E, int n_panes, int grid, hipStream_t s)
{
    if constexpr (sizeof(R) == 4)
        hipLaunchKernelGGL(k_bubbly_eval_mfma<R>, dim3(grid), dim3(kEvalBlock), 0, s, jobs, bands, w, cur, params, E,
                           n_panes);
    else
        hipLaunchKernelGGL(k_bubbly_eval_fp64, dim3(grid), dim3(kBlock), 0, s, jobs, bands, w, cur, params, E);
}
template <class R>
void launch_shade_bubbly(const JobDev *jobs, const BandDev *bands, const Work<R> &w, int cur, int grid, hipStream_t s)
{
    hipLaunchKernelGGL(k_shade_bubbly<R>, dim3(grid), dim3(kBlock), 0, s, jobs, bands, w, cur);
}
template <class R>
void launch_shadow_trace(const JobDev *jobs, const BandDev *bands, const Work<R> &w, int lds_job, bool one_job,
                         int grid, hipStream_t s)
{
    if (one_job) hipLaunchKernelGGL((k_shadow_trace<R, true>), dim3(grid), dim3(kBlock), 0, s, jobs, bands, w, lds_job);
    else hipLaunchKernelGGL((k_shadow_trace<R, false>), dim3(grid), dim3(kBlock), 0, s, jobs, bands, w, lds_job);
}
template <class R>
void launch_shadow_accum(const JobDev *jobs, const BandDev *bands, const Work<R> &w, bool one_job, int grid,
                         hipStream_t s)
{
    if (one_job) hipLaunchKernelGGL((k_shadow_accum<R, true>), dim3(grid), dim3(kBlock), 0, s, jobs, bands, w);
    else hipLaunchKernelGGL((k_shadow_accum<R, false>), dim3(grid), dim3(kBlock), 0, s, jobs, bands, w);
}

template <class R>
void launch_sig_hits(const JobDev *jobs, const BandDev *bands, const Work<R> &w, int cur, int grid, hipStream_t s)
{
    hipLaunchKernelGGL((k_sig_hits<R>), dim3(grid), dim3(kBlock), 0, s, jobs, bands, w, cur);
}

template <class R>
void launch_sig_shadow(const JobDev *jobs, const BandDev *bands, const Work<R> &w, int grid, hipStream_t s)
{
    hipLaunchKernelGGL((k_sig_shadow<R>), dim3(grid), dim3(kBlock), 0, s, jobs, bands, w);
}

template <class R>
void launch_resample(const float *tab_x, int n_tab, const float *tab_y, int rows, const float *xs, int nl,
                     int stride, R *out, hipStream_t s)
{
    const int total = rows * stride;
    const int grid = std::max(1, std::min(1024, (total + kBlock - 1) / kBlock));
    hipLaunchKernelGGL(k_resample<R>, dim3(grid), dim3(kBlock), 0, s, tab_x, n_tab, tab_y, rows, xs, nl, stride,
                       out);
}

void launch_finalize(const double *acc, int64_t npix, int nl, int spp, const double *wts, const double *cmf,
                     float *spec, double *xyz, hipStream_t s)
{
    const int grid = (int)std::max<int64_t>(1, std::min<int64_t>(8192, (npix + 3) / 4));   // 4 pixels per block
    hipLaunchKernelGGL(k_finalize, dim3(grid), dim3(kBlock), 0, s, acc, npix, nl, spp, wts, cmf, spec, xyz);
}
void launch_zero_f64(double *a, int64_t n, hipStream_t s)
{
    const int grid = (int)std::max<int64_t>(1, std::min<int64_t>(16384, (n + kBlock - 1) / kBlock));
    hipLaunchKernelGGL(k_zero_f64, dim3(grid), dim3(kBlock), 0, s, a, n);
}
void launch_advance_cursor(Counters *c, uint32_t chunk, hipStream_t s)
{
    hipLaunchKernelGGL(k_advance_cursor, dim3(1), dim3(64), 0, s, c, chunk);
}
void launch_zero_counters(Counters *c, hipStream_t s)
{
    hipLaunchKernelGGL(k_zero_counters, dim3(1), dim3(64), 0, s, c);
}
void launch_reset_records(Counters *c, hipStream_t s)
{
    hipLaunchKernelGGL(k_reset_records, dim3(1), dim3(64), 0, s, c);
}
void launch_slab_eval(int64_t m, const float *c, const float *lam, const float *d, const float *n, const float *k,
                      const float *tint, float *R, float *T, hipStream_t s)
{
    const int grid = (int)std::max<int64_t>(1, std::min<int64_t>(8192, (m + kBlock - 1) / kBlock));
    hipLaunchKernelGGL(k_slab_eval, dim3(grid), dim3(kBlock), 0, s, m, c, lam, d, n, k, tint, R, T);
}
void launch_debug_intersect(const SceneDev &sc, uint32_t m, const float *o, const float *d, const int32_t *skip,
                            const int32_t *orig_to_leaf, float *t, int32_t *tri, float *uv,
                            int32_t *gstack, int grid, hipStream_t s)
{
    hipLaunchKernelGGL(k_debug_intersect, dim3(grid), dim3(kBlock), 0, s, sc, m, o, d, skip, orig_to_leaf, t, tri,
                       uv, gstack);
}
void launch_debug_shadow(const SceneDev &sc, uint32_t m, const float *o, const int32_t *skip,
                         const int32_t *orig_to_leaf, float lambda_nm, const float *n_at, const float *k_at,
                         const float *t_at, float *T, int32_t *gstack, int grid, hipStream_t s)
{
    hipLaunchKernelGGL(k_debug_shadow, dim3(grid), dim3(kBlock), 0, s, sc, m, o, skip, orig_to_leaf, lambda_nm, n_at,
                       k_at, t_at, T, gstack);
}

int block_size() { return kBlock; }
int trace_block_size() { return kTraceBlock; }

// Resident blocks per CU of each render kernel: every pass is launched with
// exactly the blocks the chip holds at once, so no block waits for a second
// round while the others idle.
template <class R>
int occupancy(int kernel_class, int lds_bytes)
{
    const void *f = nullptr;
    switch (kernel_class) {
    case SDM_K_TRACE: f = (const void *)k_trace<R, true, false>; break;
    case SDM_K_SHADE: f = (const void *)k_shade<R, false>; break;
    case SDM_K_SHADE_GLASS: f = (const void *)k_shade_glass<R, false>; break;
    case SDM_K_BUBBLY_EVAL:
        if constexpr (sizeof(R) == 4) f = (const void *)k_bubbly_eval_mfma<R>;
        else f = (const void *)k_bubbly_eval_fp64;
        break;
    case SDM_K_SHADE_BUBBLY: f = (const void *)k_shade_bubbly<R>; break;
    case SDM_K_SHADOW: f = (const void *)k_shadow_trace<R, false>; break;
    case SDM_K_SHADOW_ACCUM: f = (const void *)k_shadow_accum<R, false>; break;
    default: return 1;
    }
    int b = 0;
    const int threads = kernel_class == SDM_K_SHADE ? kShadeBlock
                        : kernel_class == SDM_K_TRACE ? kTraceBlock
                        : (kernel_class == SDM_K_BUBBLY_EVAL && sizeof(R) == 4) ? kEvalBlock
                                                                                : kBlock;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&b, f, threads, lds_bytes) != hipSuccess) return 1;
    return std::max(1, b);
}

#define SDM_INSTANTIATE(R)                                                                                         \
    template void launch_generate<R>(const JobDev *, const BandDev *, const ItemDev *, int, const Work<R> &,       \
                                     uint64_t, uint32_t, int, hipStream_t);                                        \
    template void launch_trace<R>(const JobDev *, const Work<R> &, int, int, bool, bool, int, hipStream_t);        \
    template void launch_dd_trace<R>(const JobDev *, const Work<R> &, int, bool, int, bool, int, hipStream_t);    \
    template void launch_photon_pass<R>(const JobDev *, const PhotonWork<R> &, int, int, hipStream_t);            \
    template void launch_caustic<R>(const JobDev *, const BandDev *, const Work<R> &, const PhotonWork<R> &, int,  \
                                    hipStream_t);                                                                 \
    template void launch_shade<R>(const JobDev *, const BandDev *, const Work<R> &, int, bool, int, hipStream_t);  \
    template void launch_shade_glass<R>(const JobDev *, const BandDev *, const Work<R> &, int, bool, int,          \
                                        hipStream_t);                                                              \
    template void launch_bubbly_eval<R>(const JobDev *, const BandDev *, const Work<R> &, int, const float *,      \
                                        const float *, int, int, hipStream_t);                                     \
    template void launch_shade_bubbly<R>(const JobDev *, const BandDev *, const Work<R> &, int, int, hipStream_t); \
    template void launch_shadow_trace<R>(const JobDev *, const BandDev *, const Work<R> &, int, bool, int, hipStream_t); \
    template void launch_shadow_accum<R>(const JobDev *, const BandDev *, const Work<R> &, bool, int, hipStream_t); \
    template void launch_resample<R>(const float *, int, const float *, int, const float *, int, int, R *,         \
                                     hipStream_t);                                                                 \
    template void launch_sig_hits<R>(const JobDev *, const BandDev *, const Work<R> &, int, int, hipStream_t);     \
    template void launch_sig_shadow<R>(const JobDev *, const BandDev *, const Work<R> &, int, hipStream_t);       \
    template int occupancy<R>(int, int);

SDM_INSTANTIATE(float)
SDM_INSTANTIATE(double)

}  // namespace sdm
