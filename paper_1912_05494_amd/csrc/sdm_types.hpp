// sdm_types.hpp -- data layouts shared by the host runtime and the kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace sdm {

// Wide BVH node: the boxes of up to four children in SoA order (so one node
// fetch tests four boxes with vector-friendly loads) and, per child, a
// traversal entry: an inner-node index (>= 0), a leaf -1 - (first << 8 |
// count) (<= -2), or kNoChild.  Nodes are stored breadth-first so the top
// levels are an index prefix that kernels stage in LDS.  128 bytes, one
// cache line; the last 16 bytes are padding.
constexpr int32_t kNoChild = -1;
struct alignas(128) BvhNode {
    float lox[4], hix[4], loy[4], hiy[4], loz[4], hiz[4];
    int32_t child[4];
    int32_t pad[4];
};
static_assert(sizeof(BvhNode) == 128, "node layout");

// Triangle in BVH leaf order: the three vertices (exact float inputs, edges
// are formed in the kernel's precision); a.w, b.w and c.w hold, as integer
// bits, the caller's triangle index, the material index and the material's
// type (0 Lambert, 1 glass, 2 bubbly glass, 3 gray Lambert).
struct alignas(16) TriDev {
    float4 a, b, c;
};

// Candidate of the sun grid: a copy of the triangle's vertices (the exact
// floats of TriDev, so the triangle test gives the same result) with, in the
// w words, its leaf index (integer bits), its largest depth along the sun
// direction and its material type (integer bits).  A ray reads its cell's
// candidates as one contiguous stream, with no dependent loads.
struct alignas(16) GridCand {
    float4 a;   // vertex 0, leaf
    float4 b;   // vertex 1, largest depth
    float4 c;   // vertex 2, material type | material index << 2
};

// Scene data resident on the device.
// Geometric sub-domains (Sec. 5): a grid of cells over the scene's bounds,
// each with its own 4-wide BVH over the triangles that overlap it.  The
// cells' triangles are copies (a.w the caller's index, b.w the material, c.w
// the material type) in each cell's leaf order; leaf maps a copy back to the
// scene's leaf-order triangle.
struct CellDev {
    float lo[3], hi[3];
    int32_t node_base, tri_base;    // into DdDev::nodes, and DdDev::tris / leaf
    int32_t n_nodes, n_tris;
};
struct DdDev {
    int32_t n[3], n_cells;          // cells along x, y, z (n_cells = 0: no sub-domains)
    float lo[3], size[3];           // grid origin and cell extent
    int32_t sweeps;                 // passes per bounce: a multiple of 3, >= n[0] + n[1] + n[2]
    int32_t march;                  // 1: a ray goes on into the next cell in the same thread
    const CellDev *cells;
    const BvhNode *nodes;
    const TriDev *tris;
    const int32_t *leaf;
};

struct SceneDev {
    const BvhNode *nodes;
    const TriDev *tris;
    // [3][rot_n]: copy k of tris with each vertex p stored as (p[k + 1],
    // p[k + 2], p[k]) (indices mod 3), the frame of the FP32 triangle test of
    // rays whose dominant axis is k; w words as in tris
    const TriDev *tris_rot;
    int32_t rot_n;
    const float4 *thick;        // per leaf-order triangle: vertex thickness (mm)
    const int32_t *mat_type;    // [n_mat]: 0 Lambert, 1 glass, 2 bubbly glass, 3 gray Lambert
    const float *mat_thick;     // [n_mat] default thickness
    const double *mat_bub;      // [n_mat][4]: bubble extinction (per mm), inner index n_ref,
                                // density (per mm^3), pane type; zeros for other materials
    int32_t n_nodes, nt, n_mat, has_vthick;
    float sun[3];
    // sun grid (shadow rays): the point o projects to (o.e1, o.e2); cell
    // (floor((a - u0) idu), floor((b - v0) idv)) lists its candidates in
    // g_cand[g_start[c] .. g_start[c + 1]) by increasing smallest depth o.sun
    const int32_t *g_start;
    const GridCand *g_cand;
    const GridCand *g_cand_rot;   // g_cand with vertices rotated by g_rot, the sun's dominant axis
    int32_t g_rot;
    float g_e1[3], g_e2[3], g_u0, g_v0, g_idu, g_idv, g_marg;
    int32_t g_nx, g_ny, g_use;
    float teps_f;
    double teps_d;
    // distribution maps (n_maps = 0: none): per material the map index or
    // -1; per map (W, H, first texel, has thickness); texel materials and
    // thicknesses; per leaf-order triangle its vertices' texture coordinates
    // (s0, t0, s1, t1), (s2, t2, 0, 0)
    const int32_t *mat_map;
    const int4 *map_hdr;
    const int32_t *map_mat;
    const float *map_thick;
    const float4 *tri_uv;
    int32_t n_maps;
    DdDev dd;
};

// One render job (an image of one scene).  Spectral tables are in the
// kernel precision at the job's render wavelengths, [n_mat][nl] row-major.
struct JobDev {
    SceneDev sc;
    double eye[3], f[3], r[3], u[3];
    double th, aspect, oh;
    int32_t projection, W, H, spp, nl, max_depth;
    uint64_t seed;
    uint32_t job_word;
    int32_t ms;                 // row stride of the wavelength tables: nl rounded up to 4
    uint64_t acc_off;           // offset of this job's accumulator (doubles)
    const void *rho, *n, *k, *tint, *E, *Lsky, *lam;   // rows of ms values, 16-byte aligned
    double beta_thr;
    // bubbly panes
    int32_t btdf_mode;          // kBtdfExact, kBtdfSurrogate or kBtdfFallback
    int32_t err_dims[3];        // error-table cells along cos, thickness, density
    const float *err_table;     // [n_panes][err_dims] (fallback mode)
    float err_bound;            // a cell above this uses the exact walk
    // caustic photon map (photon mapping, Sec. 3.2)
    int32_t caustic;            // 1: every Lambert vertex keeps a record for the gather
    int32_t pad1;
};

constexpr uint32_t kPhotonTag = 0xFFFFFFF0u;
constexpr uint32_t kPhCoarseBits = 1u << 16, kPhCoarseWords = kPhCoarseBits / 32;   // 8 KiB, staged in LDS   // sample word of photon draws (camera samples stay below 2^31)

// A photon of the caustic map, at rest on a Lambert surface: position, the
// normal of the side it arrived on, its wavelength index and power.
template <class R>
struct alignas(16) PhotonRec {
    R x, y, z, phi;
    R nx, ny, nz;
    int32_t j;
};

constexpr int kBtdfExact = 0, kBtdfSurrogate = 1, kBtdfFallback = 2;
constexpr float kLambdaRef = 560.0f;   // wavelength of a bubbly pane's inner index and lobe width

// Spectral band (sub-domain): wavelengths [l0, l0 + nb) of a job.
struct BandDev {
    int32_t job, l0, nb, pad;
};

// Work item: a band x pixel tile x sample range; rays of an item are
// numbered pixel-major, sample-minor, starting at `first`.
struct ItemDev {
    int32_t band, x0, y0, tw, th, s0, ns, pad;
    uint64_t first;
};

// Device counters.  Kernels clear the counters the next kernel needs (never
// a memset), so a captured launch sequence replays cleanly.
// Each counter that waves update concurrently sits in a 256-byte line of
// its own, so atomics on different counters do not serialise on one line.
constexpr int kCounterPad = 64;   // 32-bit words per line
struct alignas(256) Counters {
    uint32_t count[2];          // paths in pool 0 / pool 1 (only count[cur ^ 1] is updated in a pass)
    uint32_t pad_c[kCounterPad - 2];
    uint32_t scount;            // shadow records
    uint32_t pad_s[kCounterPad - 1];
    uint32_t gcount;            // glass vertices queued for the glass shading pass
    uint32_t pad_g[kCounterPad - 1];
    uint32_t bcount;            // bubbly-glass vertices, queued from the back of gidx
    uint32_t pad_b[kCounterPad - 1];
    uint32_t kcount;            // sky records (escaped paths), from the back of the record buffer
    uint32_t pad_k[kCounterPad - 1];
    uint32_t ddn[3];            // sub-domain interface queues: entries (see k_dd_sweep)
    uint32_t pad_d[kCounterPad - 3];
    uint32_t phcount;           // photons stored in the caustic map
    uint32_t pad_p[kCounterPad - 1];
    uint32_t overflow;          // bit 0: a pool or record buffer was full;
                                // bit 1: a shadow ray crossed more than kMaxGlass panes;
                                // bit 2: a ray crossed more sub-domains than the sweeps cover
    int32_t lds_job;            // job whose BVH prefix the traversal kernels stage in LDS
    unsigned long long r0;      // first primary path of the current chunk (advanced per chunk)
    unsigned long long closest, shadow, forks, bubbly;
    unsigned long long spec_paths, spec_records;   // kSpectral paths shaded / shadow records made
    unsigned long long glass[2];   // glass vertices shaded [all, arriving with per-wavelength factors]
    unsigned long long nodes[2], tris[2];   // traversal work [closest, shadow]
    unsigned long long interface_rays;      // rays handed from a sub-domain to its neighbour
};

// Per-wavelength arrays are slot-major: the nb_max values of a slot are
// contiguous (nb_max is a multiple of 4, so every row is 16-byte aligned).
// The per-wavelength factors are touched only at sparse slots (glass
// vertices, spectral paths and records), so each lane reads and writes one
// contiguous row rather than a word in every 64-slot block.
__host__ __device__ __forceinline__ size_t aosoa(uint32_t slot, int j, int nbmax)
{
    return (size_t)slot * (size_t)nbmax + (size_t)j;
}

// Path pool (SoA).  Two pools alternate: shade reads one and writes the
// survivors, compacted, into the other.
// Path weights are factored: beta_j = g * b_j.  A path whose wavelengths all
// carry the same weight (camera rays, bounces on gray materials) keeps only
// the scalar g; the per-wavelength factors b_j exist once glass or a coloured
// material has made the weights differ, which kSpectral in its sample word
// records.  Shadow records likewise: contribution_j = scs * E_j * c_j with the
// c_j stored only for records flagged kSpectral in their pixel word.
constexpr uint32_t kSpectral = 0x80000000u;

// A path's state as three 16-byte records per slot (32-byte ones in FP64), so
// that each is moved with one wide access and a pass reads only those it
// needs: the origin with the last triangle hit, the direction, and the
// sample words with the scalar factor.
template <class R>
struct alignas(16) PathO {
    R x, y, z;
    int32_t skip;               // leaf-order index of the last hit triangle (-1: none)
};
template <class R>
struct alignas(16) PathD {
    R x, y, z;
};
template <class R>
struct alignas(16) PathS {
    uint32_t pix, smp, aux;     // smp: sample | kSpectral; aux = depth | band << 8 | job << 20
    R g;                        // scalar factor of the weights
};

template <class R>
struct Pool {
    PathO<R> *o;
    PathD<R> *d;
    PathS<R> *s;
    R *beta;                    // AoSoA [slot][j] per-wavelength factors (kSpectral paths)
};

constexpr int kMaxGlass = 8;    // panes a shadow ray may cross (more: SDM_E_UNSUPPORTED)

// Closest hit of a pool slot (tri < 0: no hit), one record so that it is
// written and read with one or two 16-byte accesses.
// A ray handed across a sub-domain interface: its pool slot, the cell it
// enters and the ray parameter where it enters (Sec. 5: the ray's state is
// continuous across the interface; origin and direction stay in the pool).
template <class R>
struct alignas(16) DdEntry {
    R t;
    uint32_t slot;
    int32_t cell;
};

template <class R>
struct alignas(16) HitRec {
    R t, u, v;                  // distance and barycentric coordinates
    int32_t tri;                // leaf-order index of the triangle hit
};

// A clear-glass vertex as the shade pass queues it for the glass pass: the
// state the glass pass needs, gathered into one record (64 bytes in FP32)
// so that it is read with a few wide loads instead of a word from each pool
// array at a scattered slot.
template <class R>
struct alignas(16) GlassRec {
    R x[3];                     // hit point
    R d[3];                     // incoming direction
    R g, u, v;                  // scalar factor; barycentric coordinates of the hit
    int32_t tri;                // leaf-order index of the pane triangle
    uint32_t aux, pix, smp;     // as in the pool
    uint32_t slot;              // pool slot (its per-wavelength factors)
};

template <class R>
struct Work {
    Pool<R> p[2];
    HitRec<R> *hit;             // closest hit per slot of the current pool
    DdEntry<R> *ddq[2];         // sub-domain interface queues (ping-pong)
    uint32_t *gidx;             // slots of the current pool at a bubbly-glass vertex, from the
                                // back: gidx[cap - 1 - b]
    GlassRec<R> *grec;          // clear-glass vertices [0, gcount)
    R *bratio;                  // AoSoA [slot][j]: surrogate R / (R + T) at bubbly vertices
    R *bw;                      // [slot]: surrogate lobe width at kLambdaRef
    R *sx, *sy, *sz;            // shadow records [0, scount); sky records of escaped paths at
                                // cap - 1 - k, k < kcount (pixel, aux, scalar and spectral factors only)
    int32_t *sskip;
    uint32_t *spix, *saux;      // spix: pixel | kSpectral
    R *scs;                     // [record] scalar factor of the contributions
    R *sgr;                     // [record] g rho / pi without the sun's cosine (caustic gather)
    R *snx, *sny, *snz;         // [record] normal on the side the path arrived (caustic gather)
    R *contrib;                 // AoSoA [record][j] per-wavelength factors (kSpectral records)
    int32_t *socc;              // panes crossed (0..kMaxGlass), -1 occluded
    int32_t *sg_leaf;           // [record][kMaxGlass] panes crossed, and at each crossing
    R *sg_d;                    //   the pane's thickness and
    int32_t *sg_m;              //   its material (distribution maps resolved)
    double *acc;
    Counters *cnt;
    uint32_t cap;               // slots of each pool and of the record buffer
    int32_t nbmax;              // row length of the per-wavelength arrays (band size rounded up to 4)
    int32_t *gstack;            // traversal stack overflow (global)
    int32_t *gstack_sh;         // the shadow walk's own (it may run beside the closest-hit pass)
    unsigned long long *sig;    // event signatures per accumulator entry (debug), or null
};

constexpr int kAuxDepthBits = 8;
constexpr int kAuxBandShift = 8;
constexpr int kAuxBandBits = 12;
constexpr int kAuxJobShift = 20;
constexpr int kMaxBand = 128;
constexpr int kLdsStack = 8;       // traversal stack levels held in LDS; deeper ones in global memory
constexpr int kMaxBvhDepth = 62;   // depth cap of the binary tree the wide nodes are collapsed from
constexpr int kMaxLeafTris = 255;  // leaf size bound of the stack encoding
constexpr int kMaxTris = 1 << 23;  // triangles per scene (stack encoding)

__host__ __device__ inline uint32_t pack_aux(int depth, int band, int job)
{
    return (uint32_t)depth | ((uint32_t)band << kAuxBandShift) | ((uint32_t)job << kAuxJobShift);
}

// The photon pass's buffers and emission square (see k_photon).
template <class R>
struct PhotonWork {
    uint32_t n;                     // photons shot
    uint32_t cap;                   // photons that can be stored
    uint32_t mask;                  // hash buckets - 1
    uint32_t nblk;                  // scan blocks
    PhotonRec<R> *rec, *sorted;
    uint32_t *start;                // [buckets + 1]: counts, then first photon of each bucket
    uint32_t *cursor;               // [buckets]
    uint32_t *part;                 // [nblk] scan block sums
    uint32_t *occ;                  // occupancy bits: bit (b & occ_mask) set when bucket b holds a photon
    uint32_t occ_mask;              // occupancy bits - 1 (a power of two, at least 32)
    uint32_t *cocc;                 // [kPhCoarseWords] coarse occupancy: cells of side 3 r, hashed
    int32_t *gstack;
    Counters *cnt;
    double r;                       // cell side and gather radius
    double lo[3];                   // hash grid origin
    double c[3], e1[3], e2[3];      // emission square: centre and half-side axes
    double power;                   // E(lambda) factor: square area x wavelengths / photons
};

}  // namespace sdm
