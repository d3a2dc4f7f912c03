// runtime.hpp -- host-side objects behind the C ABI handles (context, scene,
// network) and the error helpers shared by the API translation units.
#pragma once
#include <hip/hip_runtime.h>
#include <atomic>

#include <algorithm>
#include <string>
#include <vector>

#include "../../include/sdm.h"
#include "sdm_types.hpp"

namespace sdm_rt {

// FNV-1a (64-bit) over byte ranges: identifies a render's inputs in a
// checkpoint header.
struct Digest {
    uint64_t h = 1469598103934665603ull;
    void add(const void *p, size_t n)
    {
        const unsigned char *b = static_cast<const unsigned char *>(p);
        for (size_t i = 0; i < n; ++i) {
            h ^= b[i];
            h *= 1099511628211ull;
        }
    }
    template <class T> void add_value(const T &v) { add(&v, sizeof(v)); }
};

// Allocation-failure injection for tests of the error paths: a positive
// count n makes the n-th device allocation from then on fail as out of
// memory, once (set from SDM_FAIL_ALLOC at sdm_context_create).
inline std::atomic<long> &fail_alloc_countdown()
{
    static std::atomic<long> c{0};
    return c;
}

struct DevBuf {
    void *p = nullptr;
    size_t bytes = 0;
    hipError_t ensure(size_t b)
    {
        if (b <= bytes && p) return hipSuccess;
        release();
        if (fail_alloc_countdown().load() > 0 && fail_alloc_countdown().fetch_sub(1) == 1) return hipErrorOutOfMemory;
        hipError_t e = hipMalloc(&p, std::max<size_t>(b, 256));
        if (e != hipSuccess) { p = nullptr; bytes = 0; return e; }
        bytes = std::max<size_t>(b, 256);
        return hipSuccess;
    }
    void release()
    {
        if (p) (void)hipFree(p);
        p = nullptr;
        bytes = 0;
    }
    template <class T> T *as() const { return reinterpret_cast<T *>(p); }
    ~DevBuf() { release(); }
};

}  // namespace sdm_rt

using sdm_rt::DevBuf;

struct sdm_context {
    int device = 0;
    int num_cu = 0;
    std::string err;
    DevBuf gstack;
    // render work buffers (one set; reallocated when a render needs more)
    DevBuf pool, hits, shadowq, acc, counters, jobs, bands, items, tables, outs;
    sdm::Counters *host_counters = nullptr;
    std::vector<hipEvent_t> events;
    DevBuf slab_tmp;
    DevBuf mc_acc, flag;
    double *mc_scratch = nullptr;   // the device's static scratch (sdm_slab_mc_noalloc)
    DevBuf bubq, errtab;        // surrogate branch ratios and lobe widths; error table
    // graph replay of a chunk's kernel sequence (on a stream of the context,
    // default priority), cached while its launch arguments stay the same
    hipStream_t gstream = nullptr;
    hipEvent_t join[2] = {nullptr, nullptr};
    // the second stream of a chunk's sequence: a bounce's shadow walk and
    // accumulation run on it beside the next bounce's closest-hit pass
    // (default priority); fork / rejoin order the two streams
    hipStream_t side = nullptr;
    hipEvent_t fork = nullptr, rejoin = nullptr;
    bool overlap = true;        // false with SDM_SERIAL=1 at context creation
    hipGraphExec_t gexec = nullptr;
    std::vector<unsigned char> gkey;
    // event signatures of a render (debug; sized like acc)
    DevBuf sig;
    // partial render after SDM_E_ABORTED: its accumulator stays in acc
    struct Partial {
        bool valid = false;
        uint64_t digest = 0;          // render_digest of the scene and parameters
        int32_t tw = 0, th = 0;       // resolved pixel tile
        std::vector<uint8_t> done;    // per work item, in plan order
        size_t acc_elems = 0;         // doubles of the accumulator
    } partial;
    DevBuf acc_base;                  // the accumulator a resumed render starts from
    DevBuf ph_rec, ph_sorted, ph_start, ph_cursor, ph_part, ph_occ, ph_cocc;   // caustic photon map
    // autotuned (chunk, tile, traversal blocks per CU) per scene and render shape
    struct Tuned {
        const sdm_scene *scene;
        int32_t W, H, nl, depth, precision;
        int64_t chunk;
        int32_t tw, th;
        int32_t trace_bpc, shadow_bpc;
    };
    std::vector<Tuned> tuned;
};

struct sdm_mlp {
    sdm_context *ctx = nullptr;
    int32_t n_panes = 0;
    int64_t P = 0;
    int64_t t = 0;   // Adam steps taken
    DevBuf params, m1, m2, wb, bb, partial, loss_partial, loss;
};

struct sdm_scene {
    sdm_context *ctx = nullptr;
    sdm::SceneDev dev{};
    DevBuf nodes, tris, thick, mat_type, mat_thick, mat_bub, orig_to_leaf, tab_x, tab_mat, tab_sun, tab_sky;
    DevBuf tris_rot;            // tris rotated into the three frames of the FP32 triangle test
    DevBuf g_start, g_cand, g_cand_rot;   // sun grid (empty when shadow rays walk the BVH)
    DevBuf mat_map, map_hdr, map_mat, map_thick, tri_uv;   // distribution maps
    DevBuf dd_cells, dd_nodes, dd_tris, dd_leaf;           // geometric sub-domains
    int32_t dd_n[3] = {1, 1, 1};
    int64_t dd_refs = 0, dd_nodes_n = 0;                   // triangle references and nodes of the cells
    int32_t dd_stack = 0;
    int64_t grid_cells = 0, grid_cands = 0;
    int32_t n_tab = 0, n_mat = 0, depth = 0, n_nodes = 0, nt = 0;
    int32_t stack = 0;          // most traversal stack entries a walk can hold
    int32_t max_pane = -1;      // largest pane type of a bubbly material (-1: none)
    double lo[3] = {0, 0, 0}, hi[3] = {0, 0, 0};   // bounds of the triangles
    uint64_t digest = 0;        // of the scene description's inputs
};

namespace sdm_rt {

// Records the message of a failure in the context and returns code.
int fail(sdm_context *ctx, int code, const char *fmt, ...);
bool ptr_is_device(const void *p);

#define HIPCHK(ctx, x)                                                                            \
    do {                                                                                          \
        hipError_t e_ = (x);                                                                      \
        if (e_ != hipSuccess)                                                                     \
            return ::sdm_rt::fail(ctx, e_ == hipErrorOutOfMemory ? SDM_E_NOMEM : SDM_E_DEVICE,    \
                                  "%s: %s", #x, hipGetErrorString(e_));                           \
    } while (0)

template <class T>
hipError_t upload(DevBuf &b, const T *src, size_t n, hipStream_t s = nullptr)
{
    hipError_t e = b.ensure(n * sizeof(T));
    if (e != hipSuccess || n == 0) return e;
    return hipMemcpyAsync(b.p, src, n * sizeof(T), hipMemcpyHostToDevice, s);
}

}  // namespace sdm_rt
