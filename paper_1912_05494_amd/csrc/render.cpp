// render.cpp -- the render runtime behind sdm_render: work planning (spectral
// bands x pixel tiles, Sec. 4 and 5), per-render tables, the wavefront chunk
// loop and its kernel sequence.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <vector>

#include "../../include/sdm.h"
#include "bvh_build.hpp"
#include "runtime.hpp"
#include "sdm_types.hpp"
#include "surrogate.hpp"
#include "wavefront.hpp"

using namespace sdm;
using namespace sdm_rt;

// ---------------------------------------------------------------------------
// Render
// ---------------------------------------------------------------------------
namespace {

struct Plan {
    std::vector<BandDev> bands;
    std::vector<ItemDev> items;
    uint64_t total_rays = 0;
    int nbmax = 0;
};

int plan_work(sdm_context *ctx, const sdm_render_params *p, int job, int tw, int th, Plan &plan)
{
    const int nl = p->n_lambda;
    std::vector<int> edges;
    if (p->band_edges) {
        edges.assign(p->band_edges, p->band_edges + p->n_bands + 1);
        if (edges.front() != 0 || edges.back() != nl)
            return fail(ctx, SDM_E_INVALID, "band_edges must start at 0 and end at n_lambda");
        for (int b = 0; b < p->n_bands; ++b)
            if (edges[b + 1] <= edges[b]) return fail(ctx, SDM_E_INVALID, "band_edges must increase");
    } else {
        // contiguous bands, the first nl mod B one wavelength larger
        const int B = p->n_bands, base = nl / B, extra = nl % B;
        edges.push_back(0);
        for (int b = 0; b < B; ++b) edges.push_back(edges.back() + base + (b < extra ? 1 : 0));
    }
    const int b0 = (int)plan.bands.size();
    for (size_t b = 0; b + 1 < edges.size(); ++b) {
        const int nb = edges[b + 1] - edges[b];
        if (nb > kMaxBand) return fail(ctx, SDM_E_UNSUPPORTED, "a band holds %d > %d wavelengths", nb, kMaxBand);
        plan.bands.push_back(BandDev{job, edges[b], nb, 0});
        plan.nbmax = std::max(plan.nbmax, nb);
    }
    if ((int)plan.bands.size() >= (1 << kAuxBandBits)) return fail(ctx, SDM_E_UNSUPPORTED, "too many bands");
    const int W = p->camera.W, H = p->camera.H;
    for (int y0 = 0; y0 < H; y0 += th)
        for (int x0 = 0; x0 < W; x0 += tw)
            for (int b = b0; b < (int)plan.bands.size(); ++b) {
                ItemDev it{};
                it.band = b;
                it.x0 = x0;
                it.y0 = y0;
                it.tw = std::min(tw, W - x0);
                it.th = std::min(th, H - y0);
                it.s0 = 0;
                it.ns = p->spp;
                it.first = plan.total_rays;
                plan.total_rays += (uint64_t)it.tw * it.th * it.ns;
                plan.items.push_back(it);
            }
    return SDM_OK;
}

int validate_params(sdm_context *ctx, const sdm_render_params *p)
{
    if (!p) return fail(ctx, SDM_E_INVALID, "null render parameters");
    const sdm_camera &c = p->camera;
    if (c.W < 1 || c.H < 1 || (int64_t)c.W * c.H > (1ll << 31))
        return fail(ctx, SDM_E_INVALID, "image size %d x %d out of range", c.W, c.H);
    if (p->spp < 1 || p->spp > 65535) return fail(ctx, SDM_E_INVALID, "spp must be in [1, 65535]");
    if (p->max_depth < 1 || p->max_depth > 255) return fail(ctx, SDM_E_INVALID, "max_depth must be in [1, 255]");
    if (p->n_lambda < 1 || !p->lambda_nm) return fail(ctx, SDM_E_INVALID, "need n_lambda >= 1 wavelengths");
    if (p->n_bands < 1 || p->n_bands > p->n_lambda)
        return fail(ctx, SDM_E_INVALID, "n_bands must be in [1, n_lambda]");
    if (c.projection != SDM_PINHOLE && c.projection != SDM_ORTHO)
        return fail(ctx, SDM_E_INVALID, "unknown projection");
    if (p->precision != SDM_PREC_FP32 && p->precision != SDM_PREC_FP64)
        return fail(ctx, SDM_E_INVALID, "unknown precision");
    if (p->btdf_mode != SDM_BTDF_EXACT && p->btdf_mode != SDM_BTDF_SURROGATE && p->btdf_mode != SDM_BTDF_FALLBACK)
        return fail(ctx, SDM_E_INVALID, "unknown btdf_mode");
    return SDM_OK;
}

// Network and error table of the bubbly panes of a scene (none needed for
// exact walks or scenes without bubbly panes).
int validate_btdf(sdm_context *ctx, const sdm_scene *sc, const sdm_render_params *p)
{
    if (sc->max_pane < 0 || p->btdf_mode == SDM_BTDF_EXACT) return SDM_OK;
    if (!p->mlp) return fail(ctx, SDM_E_INVALID, "surrogate modes need a network (mlp)");
    if (p->mlp->ctx != ctx) return fail(ctx, SDM_E_INVALID, "the network belongs to another context");
    if (sc->max_pane >= p->mlp->n_panes)
        return fail(ctx, SDM_E_INVALID, "pane type %d is beyond the network's %d embeddings", sc->max_pane,
                    p->mlp->n_panes);
    if (p->btdf_mode == SDM_BTDF_FALLBACK) {
        if (!p->err_table) return fail(ctx, SDM_E_INVALID, "fallback mode needs an error table");
        for (int a = 0; a < 3; ++a)
            if (p->err_dims[a] < 1 || p->err_dims[a] > 1024)
                return fail(ctx, SDM_E_INVALID, "err_dims must be in [1, 1024]");
        if ((int64_t)p->err_dims[0] * p->err_dims[1] * p->err_dims[2] > (1 << 20))
            return fail(ctx, SDM_E_INVALID, "error table too large");
    }
    return SDM_OK;
}

void camera_basis(const sdm_camera &c, JobDev &jb)
{
    double f[3], r[3], u[3];
    for (int a = 0; a < 3; ++a) f[a] = (double)c.target[a] - c.eye[a];
    auto nrm = [](double *v) {
        double l = std::sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
        if (l > 0) for (int a = 0; a < 3; ++a) v[a] /= l;
    };
    nrm(f);
    const double up[3] = {c.up[0], c.up[1], c.up[2]};
    r[0] = f[1] * up[2] - f[2] * up[1];
    r[1] = f[2] * up[0] - f[0] * up[2];
    r[2] = f[0] * up[1] - f[1] * up[0];
    nrm(r);
    u[0] = r[1] * f[2] - r[2] * f[1];
    u[1] = r[2] * f[0] - r[0] * f[2];
    u[2] = r[0] * f[1] - r[1] * f[0];
    for (int a = 0; a < 3; ++a) {
        jb.eye[a] = c.eye[a];
        jb.f[a] = f[a];
        jb.r[a] = r[a];
        jb.u[a] = u[a];
    }
    jb.th = std::tan(0.5 * (double)c.vfov_deg * M_PI / 180.0);
    jb.aspect = (double)c.W / (double)c.H;
    jb.oh = 0.5 * (double)c.ortho_height;
    jb.projection = c.projection;
    jb.W = c.W;
    jb.H = c.H;
}

struct Timer {
    sdm_context *ctx;
    hipStream_t s;
    bool on;
    size_t next = 0;
    std::vector<std::pair<int, size_t>> marks;  // (kernel class, event index of start)
    hipStream_t at = nullptr;                   // stream of the open mark
    // brackets the next launch on stream on_s (default: s)
    hipError_t begin(int cls, hipStream_t on_s = nullptr)
    {
        if (!on) return hipSuccess;
        at = on_s ? on_s : s;
        if (next + 2 > ctx->events.size()) {
            for (int i = 0; i < 64; ++i) {
                hipEvent_t e;
                hipError_t r = hipEventCreate(&e);
                if (r != hipSuccess) return r;
                ctx->events.push_back(e);
            }
        }
        marks.push_back({cls, next});
        hipError_t r = hipEventRecord(ctx->events[next], at);
        next += 2;
        return r;
    }
    hipError_t end()
    {
        if (!on) return hipSuccess;
        return hipEventRecord(ctx->events[marks.back().second + 1], at);
    }
};

struct JobIn {
    const sdm_scene *sc;
    const sdm_render_params *p;
    const sdm_outputs *out;
};

// Tuned (chunk, tile) of the context for a job, or the library defaults.
void job_shape(const sdm_context *ctx, const JobIn &j, uint64_t &chunk, int &tw, int &th, int *trace_bpc = nullptr,
               int *shadow_bpc = nullptr)
{
    const sdm_render_params *p = j.p;
    chunk = p->chunk_paths > 0 ? (uint64_t)p->chunk_paths : 0;
    tw = p->tile_w;
    th = p->tile_h;
    int tb = p->trace_blocks_per_cu, sb = p->shadow_blocks_per_cu;
    if (chunk == 0 && tw <= 0 && th <= 0 && tb <= 0 && sb <= 0)
        for (const auto &t : ctx->tuned)
            if (t.scene == j.sc && t.W == p->camera.W && t.H == p->camera.H && t.nl == p->n_lambda &&
                t.depth == p->max_depth && t.precision == p->precision) {
                chunk = (uint64_t)t.chunk;
                tw = t.tw;
                th = t.th;
                tb = t.trace_bpc;
                sb = t.shadow_bpc;
            }
    if (trace_bpc) *trace_bpc = std::max(tb, 0);
    if (shadow_bpc) *shadow_bpc = std::max(sb, 0);
    if (chunk == 0) chunk = (uint64_t)1 << 23;
    if (tw <= 0) tw = 16;
    if (th <= 0) th = 16;
}

// Launch arguments of one chunk's kernel sequence; a cached graph is reused
// while they are unchanged.
template <class R>
struct ChunkArgs {
    Work<R> w;
    const JobDev *jobs;
    const BandDev *bands;
    const ItemDev *items;
    const float *params, *E;
    uint64_t total;
    uint32_t chunk;
    int32_t n_items, depth, lds_job, one_job, surr, bubbly, prec, n_panes;
    int32_t dd_sweeps;                  // > 0: closest hits by geometric sub-domains
    int32_t dd_march;                   // the hand-off stays in the thread
    int32_t caustic;                    // gather the photon map after each bounce
    PhotonWork<R> pw;
    int32_t cam_fused;          // camera rays may take the fused slab form (origins in the scene's bounds)
    int32_t grid_g, grid_t, grid_s, grid_gl, grid_e, grid_b, grid_st, grid_a;   // blocks per pass
    int32_t overlap;            // 1: shadow walk and accumulation on the side stream
};

// One chunk: generate, then per bounce the closest-hit pass, shading, the
// shadow walk and the accumulation.  With a.overlap, the shadow walk and
// accumulation of bounce i (and the caustic gather) run on the side stream
// while the closest-hit pass of bounce i + 1 runs on s: both read only what
// the shading of bounce i wrote (the paths of the next pool; the records),
// the walk has its own overflow stack, and the records' counters are reset
// on the side stream after their last reader.  The shading of bounce i + 1,
// which writes new records, waits for the side stream first.
template <class R>
void enqueue_chunk(const ChunkArgs<R> &a, hipStream_t s, hipStream_t side, hipEvent_t fork, hipEvent_t rejoin,
                   Timer *tm)
{
    const bool ov = a.overlap != 0 && side != nullptr;
    hipStream_t s2 = ov ? side : s;
    auto mark = [&](int cls, hipStream_t on) { if (tm) (void)tm->begin(cls, on); };
    auto done = [&]() { if (tm) (void)tm->end(); };
    int cur = 0;
    mark(SDM_K_GENERATE, s);
    launch_generate<R>(a.jobs, a.bands, a.items, a.n_items, a.w, a.total, a.chunk, a.grid_g, s);
    done();
    for (int dpt = 0; dpt < a.depth; ++dpt) {
        mark(SDM_K_TRACE, s);
        if (a.dd_sweeps > 0)
            launch_dd_trace<R>(a.jobs, a.w, cur, dpt > 0 || a.cam_fused != 0, a.dd_sweeps, a.dd_march != 0, a.grid_t,
                               s);
        else
            launch_trace<R>(a.jobs, a.w, cur, a.lds_job, dpt > 0 || a.cam_fused != 0, a.one_job != 0, a.grid_t, s);
        done();
        if (a.w.sig) launch_sig_hits<R>(a.jobs, a.bands, a.w, cur, a.grid_s, s);
        if (ov && dpt > 0) (void)hipStreamWaitEvent(s, rejoin, 0);   // the previous bounce's records are read
        mark(SDM_K_SHADE, s);
        launch_shade<R>(a.jobs, a.bands, a.w, cur, a.one_job != 0, a.grid_s, s);
        done();
        mark(SDM_K_SHADE_GLASS, s);
        launch_shade_glass<R>(a.jobs, a.bands, a.w, cur, a.one_job != 0, a.grid_gl, s);
        done();
        if (a.surr) {
            mark(SDM_K_BUBBLY_EVAL, s);
            launch_bubbly_eval<R>(a.jobs, a.bands, a.w, cur, a.params, a.E, a.n_panes, a.grid_e, s);
            done();
        }
        if (a.bubbly) {
            mark(SDM_K_SHADE_BUBBLY, s);
            launch_shade_bubbly<R>(a.jobs, a.bands, a.w, cur, a.grid_b, s);
            done();
        }
        if (ov) {
            (void)hipEventRecord(fork, s);
            (void)hipStreamWaitEvent(s2, fork, 0);
        }
        mark(SDM_K_SHADOW, s2);
        launch_shadow_trace<R>(a.jobs, a.bands, a.w, a.lds_job, a.one_job != 0, a.grid_st, s2);
        done();
        if (a.w.sig) launch_sig_shadow<R>(a.jobs, a.bands, a.w, a.grid_s, s2);
        mark(SDM_K_SHADOW_ACCUM, s2);
        launch_shadow_accum<R>(a.jobs, a.bands, a.w, a.one_job != 0, a.grid_a, s2);
        done();
        if (a.caustic) {
            mark(SDM_K_CAUSTIC, s2);
            launch_caustic<R>(a.jobs, a.bands, a.w, a.pw, a.grid_a, s2);
            done();
        }
        if (dpt + 1 < a.depth) launch_reset_records(a.w.cnt, s2);
        if (ov) (void)hipEventRecord(rejoin, s2);
        cur ^= 1;
    }
    if (ov) (void)hipStreamWaitEvent(s, rejoin, 0);
    launch_advance_cursor(a.w.cnt, a.chunk, s);
}

// All chunks on the context's graph stream: capture one chunk's sequence
// once (or reuse the cached graph) and launch it n_chunks times; the
// caller's stream and the graph stream are ordered by events.
template <class R>
int run_graph(sdm_context *ctx, const ChunkArgs<R> &a, uint64_t n_chunks, hipStream_t s)
{
    const unsigned char *kb = reinterpret_cast<const unsigned char *>(&a);
    std::vector<unsigned char> key(kb, kb + sizeof(a));
    if (!ctx->gexec || key != ctx->gkey) {
        if (ctx->gexec) {
            HIPCHK(ctx, hipGraphExecDestroy(ctx->gexec));
            ctx->gexec = nullptr;
        }
        hipGraph_t g = nullptr;
        HIPCHK(ctx, hipStreamBeginCapture(ctx->gstream, hipStreamCaptureModeThreadLocal));
        enqueue_chunk<R>(a, ctx->gstream, ctx->side, ctx->fork, ctx->rejoin, nullptr);
        HIPCHK(ctx, hipStreamEndCapture(ctx->gstream, &g));
        const hipError_t e = hipGraphInstantiate(&ctx->gexec, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        if (e != hipSuccess) {
            ctx->gexec = nullptr;
            return fail(ctx, SDM_E_DEVICE, "graph instantiation: %s", hipGetErrorString(e));
        }
        ctx->gkey.swap(key);
    }
    HIPCHK(ctx, hipEventRecord(ctx->join[0], s));
    HIPCHK(ctx, hipStreamWaitEvent(ctx->gstream, ctx->join[0], 0));
    for (uint64_t c = 0; c < n_chunks; ++c) HIPCHK(ctx, hipGraphLaunch(ctx->gexec, ctx->gstream));
    HIPCHK(ctx, hipEventRecord(ctx->join[1], ctx->gstream));
    HIPCHK(ctx, hipStreamWaitEvent(s, ctx->join[1], 0));
    return SDM_OK;
}

// Per-job device tables: [R: rho, n, k, tint (n_mat rows each), E, Lsky,
// lambda; rows of ms = nl rounded up to 4 values, zero padded, so a row
// position that is a multiple of 4 is 16-byte aligned][lambda float]
// [trapezoid weights double][observer double].
struct TableLayout {
    size_t off, off_lamf, off_w, off_c, end;
};

inline int table_stride(int nl) { return (nl + 3) & ~3; }

TableLayout table_layout(size_t base, int nm, int nl, size_t rsize)
{
    auto up = [](size_t x) { return (x + 255) / 256 * 256; };
    const size_t ms = (size_t)table_stride(nl);
    TableLayout t;
    t.off = up(base);
    t.off_lamf = t.off + up((4 * (size_t)nm + 3) * ms * rsize);
    t.off_w = t.off_lamf + up(nl * sizeof(float));
    t.off_c = t.off_w + up(nl * sizeof(double));
    t.end = t.off_c + 3 * nl * sizeof(double);
    return t;
}

// Item budget and resumption of a single render (max_items, checkpoints).
struct Budget {
    int64_t max_items = 0;      // 0: every item still to do
    bool resume = false;        // continue ctx->partial (the accumulator holds its sums)
    uint64_t digest = 0;        // render_digest of the job
};

// Photon pass set-up (see sdm_render_params.photons): buffers, the hash grid
// of cells of side r over the scene's bounds, and the emission square: half
// sides along e1 = normalize(h x s) and e2 = s x e1 (h = (1, 2, 3) / sqrt(14),
// s the sun direction) scaled by the bounding sphere's radius rho, centred at
// the sphere's centre plus 2 rho s, area (2 rho)^2.
template <class R>
int photon_setup(sdm_context *ctx, const JobIn &j, ChunkArgs<R> &a, hipStream_t s)
{
    (void)s;
    const sdm_scene *sc = j.sc;
    PhotonWork<R> &pw = a.pw;
    pw.n = (uint32_t)j.p->photons;
    pw.cap = pw.n;
    // At most 2^23 buckets: the bucket offsets (buckets + 1 values) are
    // scanned in blocks of 4096 and the block totals by one block of 4096,
    // which covers up to 2^24 values.  Which photons a gather finds does not
    // depend on the bucket count (the radius test drops colliding cells).
    uint32_t buckets = 1024;
    while (buckets < 2u * pw.n && buckets < (1u << 23)) buckets <<= 1;
    pw.mask = buckets - 1u;
    pw.nblk = (buckets + 1u + 4095u) / 4096u;
    HIPCHK(ctx, ctx->ph_rec.ensure((size_t)pw.cap * sizeof(PhotonRec<R>)));
    HIPCHK(ctx, ctx->ph_sorted.ensure((size_t)pw.cap * sizeof(PhotonRec<R>)));
    HIPCHK(ctx, ctx->ph_start.ensure((size_t)(buckets + 1) * sizeof(uint32_t)));
    HIPCHK(ctx, ctx->ph_cursor.ensure((size_t)buckets * sizeof(uint32_t)));
    HIPCHK(ctx, ctx->ph_part.ensure((size_t)pw.nblk * sizeof(uint32_t)));
    // one occupancy bit per bucket up to 2^20 buckets (128 KiB, resident in
    // L2); above, bit b & (2^20 - 1) stands for every bucket that shares it
    pw.occ_mask = std::min<uint32_t>(buckets, 1u << 20) - 1u;
    HIPCHK(ctx, ctx->ph_occ.ensure((size_t)(pw.occ_mask + 1u) / 8u));
    HIPCHK(ctx, ctx->ph_cocc.ensure((size_t)kPhCoarseWords * 4u));
    pw.rec = ctx->ph_rec.as<PhotonRec<R>>();
    pw.sorted = ctx->ph_sorted.as<PhotonRec<R>>();
    pw.start = ctx->ph_start.as<uint32_t>();
    pw.cursor = ctx->ph_cursor.as<uint32_t>();
    pw.part = ctx->ph_part.as<uint32_t>();
    pw.occ = ctx->ph_occ.as<uint32_t>();
    pw.cocc = ctx->ph_cocc.as<uint32_t>();
    pw.gstack = a.w.gstack;
    pw.cnt = a.w.cnt;
    pw.r = j.p->photon_radius;
    double cen[3], rad = 0.0;
    for (int q = 0; q < 3; ++q) {
        pw.lo[q] = sc->lo[q];
        cen[q] = 0.5 * (sc->lo[q] + sc->hi[q]);
        rad += 0.25 * (sc->hi[q] - sc->lo[q]) * (sc->hi[q] - sc->lo[q]);
    }
    rad = std::sqrt(rad) + 1e-6;
    double sn[3] = {sc->dev.sun[0], sc->dev.sun[1], sc->dev.sun[2]};
    const double sl = std::sqrt(sn[0] * sn[0] + sn[1] * sn[1] + sn[2] * sn[2]);
    for (double &x : sn) x /= sl;
    const double hh[3] = {0.2672612419124244, 0.5345224838248488, 0.8017837257372732};
    double e1[3] = {hh[1] * sn[2] - hh[2] * sn[1], hh[2] * sn[0] - hh[0] * sn[2], hh[0] * sn[1] - hh[1] * sn[0]};
    const double l1 = std::sqrt(e1[0] * e1[0] + e1[1] * e1[1] + e1[2] * e1[2]);
    for (double &x : e1) x /= l1;
    const double e2[3] = {sn[1] * e1[2] - sn[2] * e1[1], sn[2] * e1[0] - sn[0] * e1[2], sn[0] * e1[1] - sn[1] * e1[0]};
    for (int q = 0; q < 3; ++q) {
        pw.c[q] = cen[q] + 2.0 * rad * sn[q];
        pw.e1[q] = rad * e1[q];
        pw.e2[q] = rad * e2[q];
    }
    pw.power = 4.0 * rad * rad * (double)j.p->n_lambda / (double)std::max<uint32_t>(pw.n, 1u);
    return SDM_OK;
}

template <class R>
int render_jobs(sdm_context *ctx, const std::vector<JobIn> &jobs, sdm_stats *stats, hipStream_t s,
                const Budget &bud)
{
    const int nj = (int)jobs.size();
    const sdm_render_params *p0 = jobs[0].p;
    Plan plan;
    uint64_t chunk = 0;
    int depth = 0;
    std::vector<int64_t> acc_off(nj + 1, 0);
    int tw0 = 0, th0 = 0;
    int trace_bpc = 0, shadow_bpc = 0;   // resident blocks per CU of the traversal passes (0: default)
    for (int j = 0; j < nj; ++j) {
        uint64_t ch;
        int tw, th, tb, sb;
        job_shape(ctx, jobs[j], ch, tw, th, &tb, &sb);
        if (bud.resume) {   // the partial render's items
            tw = ctx->partial.tw;
            th = ctx->partial.th;
        }
        if (j == 0) {
            chunk = ch;
            tw0 = tw;
            th0 = th;
            trace_bpc = tb;
            shadow_bpc = sb;
        }
        if (int rc = plan_work(ctx, jobs[j].p, j, tw, th, plan)) return rc;
        depth = std::max(depth, jobs[j].p->max_depth);
        acc_off[j + 1] = acc_off[j] + (int64_t)jobs[j].p->camera.W * jobs[j].p->camera.H * jobs[j].p->n_lambda;
    }
    // Items of this call: those not done yet, in plan order, at most max_items
    // (each item's paths are numbered afresh from 0).
    const size_t n_all = plan.items.size();
    std::vector<uint8_t> done;
    if (bud.resume) {
        if (ctx->partial.done.size() != n_all || ctx->partial.acc_elems != (size_t)acc_off[nj])
            return fail(ctx, SDM_E_INVALID, "the partial render has another item plan");
        done = ctx->partial.done;
    } else {
        done.assign(n_all, 0);
    }
    if (bud.resume || bud.max_items > 0) {
        std::vector<ItemDev> sel;
        uint64_t first = 0;
        for (size_t i = 0; i < n_all; ++i) {
            if (done[i]) continue;
            if (bud.max_items > 0 && (int64_t)sel.size() >= bud.max_items) break;
            ItemDev it = plan.items[i];
            it.first = first;
            first += (uint64_t)it.tw * it.th * it.ns;
            sel.push_back(it);
            done[i] = 1;
        }
        plan.items.swap(sel);
        plan.total_rays = first;
    } else {
        std::fill(done.begin(), done.end(), 1);
    }
    uint64_t n_done = 0;
    for (uint8_t x : done) n_done += x;
    const bool complete = n_done == n_all;
    // event signatures (debug)
    bool want_sig = false;
    for (const auto &j : jobs) want_sig = want_sig || j.out->events != nullptr;
    if (want_sig && (bud.resume || bud.max_items > 0))
        return fail(ctx, SDM_E_UNSUPPORTED, "event signatures need an uninterrupted render");
    if (want_sig) HIPCHK(ctx, ctx->sig.ensure((size_t)acc_off[nj] * sizeof(uint64_t)));
    if (bud.resume) {
        // a retried attempt (pool overflow) starts again from these sums
        HIPCHK(ctx, ctx->acc_base.ensure((size_t)acc_off[nj] * sizeof(double)));
        HIPCHK(ctx, hipMemcpyAsync(ctx->acc_base.p, ctx->acc.p, (size_t)acc_off[nj] * sizeof(double),
                                   hipMemcpyDeviceToDevice, s));
    }
    // tables of every job
    std::vector<TableLayout> lay(nj);
    size_t tab_bytes = 0;
    for (int j = 0; j < nj; ++j) {
        lay[j] = table_layout(tab_bytes, jobs[j].sc->n_mat, jobs[j].p->n_lambda, sizeof(R));
        tab_bytes = lay[j].end;
    }
    HIPCHK(ctx, ctx->tables.ensure(tab_bytes));
    // network and error tables (one network per batch)
    const sdm_mlp *net = nullptr;
    bool bubbly = false, surr = false;
    size_t err_elems = 0;
    for (const auto &j : jobs) {
        if (j.sc->max_pane < 0) continue;
        bubbly = true;
        if (j.p->btdf_mode == SDM_BTDF_EXACT) continue;
        surr = true;
        if (net && net != j.p->mlp) return fail(ctx, SDM_E_INVALID, "the jobs of a batch must share one network");
        net = j.p->mlp;
        if (j.p->btdf_mode == SDM_BTDF_FALLBACK)
            err_elems += (size_t)net->n_panes * j.p->err_dims[0] * j.p->err_dims[1] * j.p->err_dims[2];
    }
    if (err_elems) HIPCHK(ctx, ctx->errtab.ensure(err_elems * sizeof(float)));
    std::vector<JobDev> jd(nj);
    size_t err_pos = 0;
    for (int j = 0; j < nj; ++j) {
        const sdm_scene *sc = jobs[j].sc;
        const sdm_render_params *p = jobs[j].p;
        const int nl = p->n_lambda, nm = sc->n_mat;
        char *tb = ctx->tables.as<char>();
        R *tR = reinterpret_cast<R *>(tb + lay[j].off);
        float *lamf = reinterpret_cast<float *>(tb + lay[j].off_lamf);
        double *wts_d = reinterpret_cast<double *>(tb + lay[j].off_w);
        double *cmf_d = reinterpret_cast<double *>(tb + lay[j].off_c);
        std::vector<double> wts(nl), cmf(3 * (size_t)nl, 0.0);
        if (nl == 1) wts[0] = 1.0;
        else
            for (int i = 0; i < nl; ++i)
                wts[i] = 0.5 * ((double)p->lambda_nm[std::min(i + 1, nl - 1)] - p->lambda_nm[std::max(i - 1, 0)]);
        if (p->cmf_xyz)
            for (size_t i = 0; i < 3 * (size_t)nl; ++i) cmf[i] = p->cmf_xyz[i];
        HIPCHK(ctx, hipMemcpyAsync(lamf, p->lambda_nm, nl * sizeof(float), hipMemcpyHostToDevice, s));
        HIPCHK(ctx, hipMemcpyAsync(wts_d, wts.data(), nl * sizeof(double), hipMemcpyHostToDevice, s));
        HIPCHK(ctx, hipMemcpyAsync(cmf_d, cmf.data(), 3 * nl * sizeof(double), hipMemcpyHostToDevice, s));
        // the host vectors must outlive the asynchronous copies
        HIPCHK(ctx, hipStreamSynchronize(s));
        const size_t ms = (size_t)table_stride(nl);
        launch_resample<R>(sc->tab_x.as<float>(), sc->n_tab, sc->tab_mat.as<float>(), 4 * nm, lamf, nl, (int)ms, tR, s);
        launch_resample<R>(sc->tab_x.as<float>(), sc->n_tab, sc->tab_sun.as<float>(), 1, lamf, nl, (int)ms,
                           tR + 4 * nm * ms, s);
        launch_resample<R>(sc->tab_x.as<float>(), sc->n_tab, sc->tab_sky.as<float>(), 1, lamf, nl, (int)ms,
                           tR + (4 * nm + 1) * ms, s);
        launch_resample<R>(lamf, nl, lamf, 1, lamf, nl, (int)ms, tR + (4 * nm + 2) * ms, s);
        JobDev &jb = jd[j];
        jb = JobDev{};
        jb.sc = sc->dev;
        camera_basis(p->camera, jb);
        jb.spp = p->spp;
        jb.nl = nl;
        jb.max_depth = p->max_depth;
        jb.seed = p->seed;
        jb.job_word = p->job_id;
        jb.acc_off = (uint64_t)acc_off[j];
        jb.ms = (int32_t)ms;
        jb.rho = tR;
        jb.n = tR + nm * ms;
        jb.k = tR + 2 * nm * ms;
        jb.tint = tR + 3 * nm * ms;
        jb.E = tR + 4 * nm * ms;
        jb.Lsky = tR + (4 * nm + 1) * ms;
        jb.lam = tR + (4 * nm + 2) * ms;
        jb.beta_thr = p->beta_threshold;
        jb.btdf_mode = p->btdf_mode;
        jb.err_bound = p->err_bound;
        jb.caustic = p->photons > 0 ? 1 : 0;
        if (sc->max_pane >= 0 && p->btdf_mode == SDM_BTDF_FALLBACK) {
            const size_t ncell = (size_t)net->n_panes * p->err_dims[0] * p->err_dims[1] * p->err_dims[2];
            HIPCHK(ctx, hipMemcpyAsync(ctx->errtab.as<float>() + err_pos, p->err_table, ncell * sizeof(float),
                                       hipMemcpyHostToDevice, s));
            HIPCHK(ctx, hipStreamSynchronize(s));
            for (int a = 0; a < 3; ++a) jb.err_dims[a] = p->err_dims[a];
            jb.err_table = ctx->errtab.as<float>() + err_pos;
            err_pos += ncell;
        }
    }
    HIPCHK(ctx, hipGetLastError());
    HIPCHK(ctx, upload(ctx->jobs, jd.data(), jd.size(), s));
    HIPCHK(ctx, upload(ctx->bands, plan.bands.data(), plan.bands.size(), s));
    HIPCHK(ctx, upload(ctx->items, plan.items.data(), plan.items.size(), s));
    HIPCHK(ctx, hipStreamSynchronize(s));

    const uint64_t total = plan.total_rays;
    chunk = std::max<uint64_t>(1, std::min<uint64_t>(chunk, std::max<uint64_t>(total, 1)));
    const bool timing = p0->timing != 0;
    const bool graph = p0->graph != 0 && !timing;
    int attempt = 0;
    for (;;) {
        // pool capacity: the chunk plus headroom for forks (doubled on overflow)
        const uint64_t cap64 = ((chunk + (chunk >> 2) * (1ull << attempt) + 1024 + 63) / 64) * 64;
        if (cap64 >= (1ull << 31)) return fail(ctx, SDM_E_NOMEM, "path pool would exceed 2^31 slots");
        const uint32_t cap = (uint32_t)cap64;
        const int nb = (plan.nbmax + 3) & ~3;   // per-wavelength row, 16-byte aligned
        const size_t plane = (size_t)cap * sizeof(R);
        const size_t pool_b = (size_t)cap * (sizeof(PathO<R>) + sizeof(PathD<R>) + sizeof(PathS<R>)) +
                              (size_t)cap * nb * sizeof(R) + 8 * 256;
        const bool dd = nj == 1 && jobs[0].sc->dev.dd.n_cells > 0;
        const size_t hit_b = (size_t)cap * sizeof(HitRec<R>) + (size_t)cap * 4 + (size_t)cap * sizeof(GlassRec<R>) +
                             (dd ? 2 * (size_t)cap * sizeof(DdEntry<R>) + 512 : 0) + 256;
        const bool caustic = nj == 1 && jobs[0].p->photons > 0;
        const size_t sh_b = (caustic ? 8 : 4) * plane + 4 * (size_t)cap * 4 + (size_t)cap * nb * sizeof(R) +
                            (size_t)cap * kMaxGlass * (8 + sizeof(R)) + 12 * 256;
        HIPCHK(ctx, ctx->pool.ensure(2 * pool_b + 1024));
        HIPCHK(ctx, ctx->hits.ensure(hit_b + 2048));
        HIPCHK(ctx, ctx->shadowq.ensure(sh_b + 2048));
        if (!bud.resume) HIPCHK(ctx, ctx->acc.ensure((size_t)acc_off[nj] * sizeof(double)));
        HIPCHK(ctx, ctx->counters.ensure(sizeof(Counters)));
        ChunkArgs<R> a{};
        const int occ_t = occupancy<R>(SDM_K_TRACE), occ_s = occupancy<R>(SDM_K_SHADOW);
        a.grid_t = ctx->num_cu * (trace_bpc > 0 ? std::min(trace_bpc, occ_t) : occ_t);
        a.grid_s = ctx->num_cu * occupancy<R>(SDM_K_SHADE);
        a.grid_gl = ctx->num_cu * occupancy<R>(SDM_K_SHADE_GLASS);
        a.grid_e = ctx->num_cu * occupancy<R>(SDM_K_BUBBLY_EVAL);
        a.grid_b = ctx->num_cu * occupancy<R>(SDM_K_SHADE_BUBBLY);
        // Sun-grid walks stream their cells' candidate lists; with five
        // resident blocks per CU the lists in flight evict each other, four
        // keep the pass faster (measured on the nave: 5.33 -> 4.93 ms)
        bool grid_walk = false;
        for (const auto &jj : jobs) grid_walk = grid_walk || jj.sc->dev.g_use != 0;
        a.grid_st = ctx->num_cu * (shadow_bpc > 0 ? std::min(shadow_bpc, occ_s) : grid_walk ? std::min(4, occ_s) : occ_s);
        a.grid_a = ctx->num_cu * occupancy<R>(SDM_K_SHADOW_ACCUM);
        a.grid_g = (int)std::max<uint64_t>(1, std::min<uint64_t>((chunk + 255) / 256, 8ull * ctx->num_cu));
        // overflow stacks: the closest-hit passes' (and the photon pass's),
        // then the shadow walk's, which may run beside them
        const size_t gt_threads = (size_t)a.grid_t * trace_block_size(), gs_threads = (size_t)a.grid_st * block_size();
        int stack = 0;
        for (const auto &jj : jobs) stack = std::max({stack, jj.sc->stack, jj.sc->dd_stack});
        const size_t levels = (size_t)global_stack_levels(stack);
        HIPCHK(ctx, ctx->gstack.ensure((gt_threads + gs_threads) * levels * sizeof(int32_t)));
        Work<R> &w = a.w;
        char *pb = nullptr;
        auto take = [&](size_t bytes) { char *r = pb; pb += (bytes + 255) / 256 * 256; return r; };
        pb = ctx->pool.as<char>();
        for (int q = 0; q < 2; ++q) {
            Pool<R> &P = w.p[q];
            P.o = (PathO<R> *)take((size_t)cap * sizeof(PathO<R>));
            P.d = (PathD<R> *)take((size_t)cap * sizeof(PathD<R>));
            P.s = (PathS<R> *)take((size_t)cap * sizeof(PathS<R>));
            P.beta = (R *)take((size_t)cap * nb * sizeof(R));
        }
        pb = ctx->hits.as<char>();
        w.hit = (HitRec<R> *)take((size_t)cap * sizeof(HitRec<R>));
        w.gidx = (uint32_t *)take((size_t)cap * 4);
        w.grec = (GlassRec<R> *)take((size_t)cap * sizeof(GlassRec<R>));
        w.ddq[0] = w.ddq[1] = nullptr;
        if (dd) {
            w.ddq[0] = (DdEntry<R> *)take((size_t)cap * sizeof(DdEntry<R>));
            w.ddq[1] = (DdEntry<R> *)take((size_t)cap * sizeof(DdEntry<R>));
        }
        if (surr) {
            HIPCHK(ctx, ctx->bubq.ensure((size_t)cap * nb * sizeof(R) + plane + 1024));
            pb = ctx->bubq.as<char>();
            w.bratio = (R *)take((size_t)cap * nb * sizeof(R));
            w.bw = (R *)take(plane);
        }
        pb = ctx->shadowq.as<char>();
        w.sx = (R *)take(plane); w.sy = (R *)take(plane); w.sz = (R *)take(plane);
        w.sskip = (int32_t *)take((size_t)cap * 4); w.spix = (uint32_t *)take((size_t)cap * 4);
        w.saux = (uint32_t *)take((size_t)cap * 4); w.socc = (int32_t *)take((size_t)cap * 4);
        w.scs = (R *)take(plane);
        w.sgr = w.snx = w.sny = w.snz = nullptr;
        if (caustic) {
            w.sgr = (R *)take(plane);
            w.snx = (R *)take(plane); w.sny = (R *)take(plane); w.snz = (R *)take(plane);
        }
        w.contrib = (R *)take((size_t)cap * nb * sizeof(R));
        w.sg_leaf = (int32_t *)take((size_t)cap * kMaxGlass * 4);
        w.sg_d = (R *)take((size_t)cap * kMaxGlass * sizeof(R));
        w.sg_m = (int32_t *)take((size_t)cap * kMaxGlass * sizeof(int32_t));
        w.acc = ctx->acc.as<double>();
        w.cnt = ctx->counters.as<Counters>();
        w.cap = cap;
        w.nbmax = nb;
        w.gstack = ctx->gstack.as<int32_t>();
        w.gstack_sh = w.gstack + gt_threads * levels;
        w.sig = want_sig ? ctx->sig.as<unsigned long long>() : nullptr;
        a.jobs = ctx->jobs.as<JobDev>();
        a.bands = ctx->bands.as<BandDev>();
        a.items = ctx->items.as<ItemDev>();
        a.n_items = (int32_t)plan.items.size();
        a.total = total;
        a.chunk = (uint32_t)chunk;
        a.depth = depth;
        a.lds_job = nj == 1 ? 0 : -2;   // a batch stages the BVH of each chunk's first job
        a.dd_sweeps = dd ? jobs[0].sc->dev.dd.sweeps : 0;
        a.dd_march = dd ? jobs[0].sc->dev.dd.march : 0;
        a.one_job = nj == 1;
        // The fused slab form's rounding stays inside the box padding for
        // origins within the scene's bounds: pinhole cameras placed inside
        // their scene may use it for the camera rays too.
        a.cam_fused = 1;
        for (const auto &jj : jobs) {
            const sdm_camera &cam = jj.p->camera;
            bool inside = cam.projection == SDM_PINHOLE && jj.sc->nt > 0;
            for (int q = 0; q < 3 && inside; ++q)
                inside = (double)cam.eye[q] >= jj.sc->lo[q] && (double)cam.eye[q] <= jj.sc->hi[q];
            if (!inside) a.cam_fused = 0;
        }
        a.surr = surr;
        // signatures read the hits a concurrent closest-hit pass would overwrite
        a.overlap = ctx->overlap && !want_sig ? 1 : 0;
        a.bubbly = bubbly;
        a.prec = sizeof(R) == 8;
        if (surr) {
            a.params = net->params.as<float>();
            a.E = net->params.as<float>() + mlp_net_params();
            a.n_panes = net->n_panes;
        }
        const uint64_t n_chunks = total == 0 ? 0 : (total + chunk - 1) / chunk;

        Timer tm{ctx, s, timing};
        hipEvent_t ev0 = nullptr, ev1 = nullptr;
        HIPCHK(ctx, hipEventCreate(&ev0));
        HIPCHK(ctx, hipEventCreate(&ev1));
        HIPCHK(ctx, hipEventRecord(ev0, s));
        if (bud.resume)
            HIPCHK(ctx, hipMemcpyAsync(w.acc, ctx->acc_base.p, (size_t)acc_off[nj] * sizeof(double),
                                       hipMemcpyDeviceToDevice, s));
        else
            launch_zero_f64(w.acc, acc_off[nj], s);
        if (want_sig) launch_zero_f64(reinterpret_cast<double *>(w.sig), acc_off[nj], s);
        launch_zero_counters(w.cnt, s);
        a.caustic = caustic ? 1 : 0;
        if (caustic) {
            if (int rc = photon_setup<R>(ctx, jobs[0], a, s)) return rc;
            (void)tm.begin(SDM_K_PHOTON);
            launch_photon_pass<R>(a.jobs, a.pw, a.grid_t, ctx->num_cu, s);
            (void)tm.end();
        }
        if (n_chunks == 0) {
            // nothing left to trace: the outputs come from the accumulator
        } else if (graph) {
            if (int rc = run_graph<R>(ctx, a, n_chunks, s)) return rc;
        } else {
            for (uint64_t c = 0; c < n_chunks; ++c)
                enqueue_chunk<R>(a, s, ctx->side, ctx->fork, ctx->rejoin, timing ? &tm : nullptr);
        }
        HIPCHK(ctx, hipGetLastError());
        // finalize every job into device outputs (or staging for host outputs)
        size_t stage_b = 0;
        for (const auto &j : jobs) {
            const size_t npix = (size_t)j.p->camera.W * j.p->camera.H;
            if (j.out->spectral && j.out->spectral_mem == SDM_MEM_HOST)
                stage_b += (npix * j.p->n_lambda * sizeof(float) + 255) / 256 * 256;
            if (j.out->xyz && j.out->xyz_mem == SDM_MEM_HOST) stage_b += (npix * 3 * sizeof(double) + 255) / 256 * 256;
        }
        if (stage_b) HIPCHK(ctx, ctx->outs.ensure(stage_b));
        size_t stage_pos = 0;
        struct Copy { void *dst; const void *src; size_t bytes; };
        std::vector<Copy> copies;
        for (int j = 0; j < nj; ++j) {
            const sdm_render_params *p = jobs[j].p;
            const sdm_outputs *out = jobs[j].out;
            const int64_t npix = (int64_t)p->camera.W * p->camera.H;
            const int nl = p->n_lambda;
            float *spec_d = nullptr;
            double *xyz_d = nullptr;
            const size_t spec_b = (size_t)npix * nl * sizeof(float), xyz_b = (size_t)npix * 3 * sizeof(double);
            if (out->spectral) {
                if (out->spectral_mem == SDM_MEM_HOST) {
                    spec_d = reinterpret_cast<float *>(ctx->outs.as<char>() + stage_pos);
                    stage_pos += (spec_b + 255) / 256 * 256;
                    copies.push_back({out->spectral, spec_d, spec_b});
                } else {
                    spec_d = out->spectral;
                }
            }
            if (out->xyz && p->cmf_xyz) {
                if (out->xyz_mem == SDM_MEM_HOST) {
                    xyz_d = reinterpret_cast<double *>(ctx->outs.as<char>() + stage_pos);
                    stage_pos += (xyz_b + 255) / 256 * 256;
                    copies.push_back({out->xyz, xyz_d, xyz_b});
                } else {
                    xyz_d = out->xyz;
                }
            }
            const char *tb = ctx->tables.as<char>();
            if (timing) HIPCHK(ctx, tm.begin(SDM_K_FINALIZE));
            launch_finalize(w.acc + acc_off[j], npix, nl, p->spp,
                            reinterpret_cast<const double *>(tb + lay[j].off_w),
                            reinterpret_cast<const double *>(tb + lay[j].off_c), spec_d, xyz_d, s);
            if (timing) HIPCHK(ctx, tm.end());
            if (out->events)
                HIPCHK(ctx, hipMemcpyAsync(out->events, w.sig + acc_off[j], (size_t)npix * nl * sizeof(uint64_t),
                                           hipMemcpyDeviceToDevice, s));
        }
        HIPCHK(ctx, hipEventRecord(ev1, s));
        HIPCHK(ctx, hipMemcpyAsync(ctx->host_counters, w.cnt, sizeof(Counters), hipMemcpyDeviceToHost, s));
        for (const auto &c : copies) HIPCHK(ctx, hipMemcpyAsync(c.dst, c.src, c.bytes, hipMemcpyDeviceToHost, s));
        HIPCHK(ctx, hipStreamSynchronize(s));
        const Counters c = *ctx->host_counters;
        if (c.overflow & 2u) {
            (void)hipEventDestroy(ev0);
            (void)hipEventDestroy(ev1);
            return fail(ctx, SDM_E_UNSUPPORTED, "a shadow ray crossed more than %d glass panes", kMaxGlass);
        }
        if (c.overflow & 4u) {
            (void)hipEventDestroy(ev0);
            (void)hipEventDestroy(ev1);
            return fail(ctx, SDM_E_DEVICE, "a ray crossed more sub-domains than the passes cover");
        }
        if (c.overflow) {
            (void)hipEventDestroy(ev0);
            (void)hipEventDestroy(ev1);
            if (++attempt > 8)
                return fail(ctx, SDM_E_DEVICE, "path pool overflow: glass forks exceed %llu slots",
                            (unsigned long long)cap64);
            continue;  // deterministic: render again with a larger pool
        }
        if (stats) {
            sdm_stats &st = *stats;
            std::memset(&st, 0, sizeof(st));
            for (const auto &j : jobs)
                st.spectral_samples += (uint64_t)j.p->camera.W * j.p->camera.H * j.p->spp * j.p->n_lambda;
            st.paths = total;
            st.closest_segments = c.closest;
            st.shadow_segments = c.shadow;
            st.forks = c.forks;
            st.bubbly_vertices = c.bubbly;
            st.spectral_paths = c.spec_paths;
            st.spectral_records = c.spec_records;
            st.glass_vertices[0] = c.glass[0];
            st.glass_vertices[1] = c.glass[1];
            st.chunks = n_chunks;
            for (int q = 0; q < 2; ++q) {
                st.nodes_visited[q] = c.nodes[q];
                st.tris_tested[q] = c.tris[q];
            }
            st.interface_rays = c.interface_rays;
            st.photons_stored = caustic ? std::min<uint64_t>(c.phcount, a.pw.cap) : 0;
            float ms = 0;
            (void)hipEventElapsedTime(&ms, ev0, ev1);
            st.ms_render = ms;
            if (tm.on)
                for (auto &mk : tm.marks) {
                    float km = 0;
                    (void)hipEventElapsedTime(&km, ctx->events[mk.second], ctx->events[mk.second + 1]);
                    st.kernel_ms[mk.first] += km;
                    st.kernel_launches[mk.first] += 1;
                }
            st.items_done = n_done;
            st.items_total = n_all;
        }
        (void)hipEventDestroy(ev0);
        (void)hipEventDestroy(ev1);
        if (bud.resume || bud.max_items > 0) {
            sdm_context::Partial &pt = ctx->partial;
            pt.valid = !complete;
            pt.digest = bud.digest;
            pt.tw = tw0;
            pt.th = th0;
            pt.done.swap(done);
            pt.acc_elems = (size_t)acc_off[nj];
            if (!complete)
                return fail(ctx, SDM_E_ABORTED, "item budget reached: %llu of %llu items done",
                            (unsigned long long)n_done, (unsigned long long)n_all);
        }
        return SDM_OK;
    }
}

int check_job(sdm_context *ctx, const JobIn &j)
{
    if (!j.sc || !j.out) return fail(ctx, SDM_E_INVALID, "null scene or outputs");
    if (j.sc->ctx != ctx) return fail(ctx, SDM_E_INVALID, "scene belongs to another context");
    if (int rc = validate_params(ctx, j.p)) return rc;
    if (int rc = validate_btdf(ctx, j.sc, j.p)) return rc;
    if (j.out->spectral && j.out->spectral_mem == SDM_MEM_DEVICE && !ptr_is_device(j.out->spectral))
        return fail(ctx, SDM_E_INVALID, "spectral output is not device memory");
    if (j.out->xyz && j.out->xyz_mem == SDM_MEM_DEVICE && !ptr_is_device(j.out->xyz))
        return fail(ctx, SDM_E_INVALID, "xyz output is not device memory");
    if (j.out->events && !ptr_is_device(j.out->events))
        return fail(ctx, SDM_E_INVALID, "events output is not device memory");
    if (j.p->max_items < 0) return fail(ctx, SDM_E_INVALID, "max_items must be >= 0");
    if (j.p->photons < 0 || j.p->photons > (int64_t)1 << 30)
        return fail(ctx, SDM_E_INVALID, "photons must be in [0, 2^30]");
    if (j.p->photons > 0 && !(j.p->photon_radius > 0.0f && std::isfinite(j.p->photon_radius)))
        return fail(ctx, SDM_E_INVALID, "photon_radius must be > 0");
    if (j.p->photons > 0 && j.p->max_items > 0)
        return fail(ctx, SDM_E_UNSUPPORTED, "the photon map is built for whole renders (no max_items)");
    return SDM_OK;
}

// Identifies a render for checkpoints: the scene's inputs and every
// parameter that decides the accumulated sums (not the observer table, which
// only enters the XYZ conversion, nor chunking, timing or graphs).
uint64_t render_digest(const sdm_scene *sc, const sdm_render_params *p)
{
    Digest dg;
    dg.add_value(sc->digest);
    const sdm_camera &c = p->camera;
    dg.add(c.eye, sizeof(c.eye));
    dg.add(c.target, sizeof(c.target));
    dg.add(c.up, sizeof(c.up));
    dg.add_value(c.vfov_deg);
    dg.add_value(c.ortho_height);
    dg.add_value(c.W);
    dg.add_value(c.H);
    dg.add_value(c.projection);
    dg.add_value(p->n_lambda);
    dg.add(p->lambda_nm, sizeof(float) * (size_t)p->n_lambda);
    dg.add_value(p->spp);
    dg.add_value(p->max_depth);
    dg.add_value(p->seed);
    dg.add_value(p->job_id);
    dg.add_value(p->n_bands);
    if (p->band_edges) dg.add(p->band_edges, sizeof(int32_t) * ((size_t)p->n_bands + 1));
    dg.add_value(p->beta_threshold);
    dg.add_value(p->precision);
    dg.add_value(p->btdf_mode);
    if (sc->max_pane >= 0 && p->btdf_mode != SDM_BTDF_EXACT) {
        dg.add_value(p->mlp);   // the network object (its weights may change between calls)
        if (p->btdf_mode == SDM_BTDF_FALLBACK) {
            dg.add(p->err_dims, sizeof(p->err_dims));
            dg.add_value(p->err_bound);
        }
    }
    return dg.h;
}

// Adds the counts and times of one render to a total (batch statistics).
void add_stats(sdm_stats &t, const sdm_stats &a)
{
    t.spectral_samples += a.spectral_samples;
    t.paths += a.paths;
    t.closest_segments += a.closest_segments;
    t.shadow_segments += a.shadow_segments;
    t.forks += a.forks;
    t.chunks += a.chunks;
    for (int q = 0; q < 2; ++q) {
        t.nodes_visited[q] += a.nodes_visited[q];
        t.tris_tested[q] += a.tris_tested[q];
        t.glass_vertices[q] += a.glass_vertices[q];
    }
    t.bubbly_vertices += a.bubbly_vertices;
    t.spectral_paths += a.spectral_paths;
    t.spectral_records += a.spectral_records;
    t.ms_render += a.ms_render;
    for (int k = 0; k < SDM_K_COUNT; ++k) {
        t.kernel_ms[k] += a.kernel_ms[k];
        t.kernel_launches[k] += a.kernel_launches[k];
    }
    t.items_done += a.items_done;
    t.items_total += a.items_total;
    t.interface_rays += a.interface_rays;
    t.photons_stored += a.photons_stored;
}

int render_any(sdm_context *ctx, const std::vector<JobIn> &jobs, sdm_stats *stats, hipStream_t s,
               const Budget &bud = Budget())
{
    const int prec = jobs[0].p->precision;
    for (const auto &j : jobs)
        if (j.p->precision != prec) return fail(ctx, SDM_E_INVALID, "the jobs of a batch must share one precision");
    HIPCHK(ctx, hipSetDevice(ctx->device));
    if (prec == SDM_PREC_FP64) return render_jobs<double>(ctx, jobs, stats, s, bud);
    return render_jobs<float>(ctx, jobs, stats, s, bud);
}

constexpr char kCkptMagic[8] = {'S', 'D', 'M', 'C', 'K', 'P', 'T', '1'};

}  // namespace

extern "C" {

int sdm_render(sdm_context *ctx, const sdm_scene *sc, const sdm_render_params *p, const sdm_outputs *out,
               void *hip_stream)
{
    if (!ctx) return SDM_E_INVALID;
    const JobIn j{sc, p, out};
    if (!p) return fail(ctx, SDM_E_INVALID, "null render parameters");
    if (int rc = check_job(ctx, j)) return rc;
    ctx->partial.valid = false;   // a new render replaces any partial one
    Budget bud;
    bud.max_items = p->max_items;
    bud.digest = render_digest(sc, p);
    return render_any(ctx, {j}, out->stats, (hipStream_t)hip_stream, bud);
}

int sdm_render_checkpoint(sdm_context *ctx, const char *path)
{
    if (!ctx) return SDM_E_INVALID;
    if (!path) return fail(ctx, SDM_E_INVALID, "null path");
    const sdm_context::Partial &pt = ctx->partial;
    if (!pt.valid) return fail(ctx, SDM_E_INVALID, "no partial render to save");
    HIPCHK(ctx, hipSetDevice(ctx->device));
    std::vector<double> acc(pt.acc_elems);
    HIPCHK(ctx, hipMemcpy(acc.data(), ctx->acc.p, acc.size() * sizeof(double), hipMemcpyDeviceToHost));
    FILE *f = std::fopen(path, "wb");
    if (!f) return fail(ctx, SDM_E_DEVICE, "cannot open %s for writing", path);
    const int64_t n_items = (int64_t)pt.done.size(), n_acc = (int64_t)pt.acc_elems;
    bool ok = std::fwrite(kCkptMagic, 1, 8, f) == 8 && std::fwrite(&pt.digest, 8, 1, f) == 1 &&
              std::fwrite(&n_items, 8, 1, f) == 1 && std::fwrite(&n_acc, 8, 1, f) == 1 &&
              std::fwrite(&pt.tw, 4, 1, f) == 1 && std::fwrite(&pt.th, 4, 1, f) == 1 &&
              std::fwrite(pt.done.data(), 1, pt.done.size(), f) == pt.done.size() &&
              std::fwrite(acc.data(), sizeof(double), acc.size(), f) == acc.size();
    ok = (std::fclose(f) == 0) && ok;
    if (!ok) return fail(ctx, SDM_E_DEVICE, "write error on %s", path);
    return SDM_OK;
}

int sdm_render_resume(sdm_context *ctx, const char *path, const sdm_scene *sc, const sdm_render_params *p,
                      const sdm_outputs *out, void *hip_stream)
{
    if (!ctx) return SDM_E_INVALID;
    if (!p || !out) return fail(ctx, SDM_E_INVALID, "null render parameters or outputs");
    const JobIn j{sc, p, out};
    if (int rc = check_job(ctx, j)) return rc;
    const uint64_t digest = render_digest(sc, p);
    const size_t n_acc = (size_t)p->camera.W * p->camera.H * p->n_lambda;
    if (path) {
        FILE *f = std::fopen(path, "rb");
        if (!f) return fail(ctx, SDM_E_INVALID, "cannot open %s", path);
        char magic[8];
        uint64_t dg = 0;
        int64_t n_items = 0, na = 0;
        int32_t tw = 0, th = 0;
        bool ok = std::fread(magic, 1, 8, f) == 8 && std::memcmp(magic, kCkptMagic, 8) == 0 &&
                  std::fread(&dg, 8, 1, f) == 1 && std::fread(&n_items, 8, 1, f) == 1 &&
                  std::fread(&na, 8, 1, f) == 1 && std::fread(&tw, 4, 1, f) == 1 && std::fread(&th, 4, 1, f) == 1;
        if (ok && (dg != digest || na != (int64_t)n_acc || n_items < 1 || n_items > (1ll << 31) || tw < 1 || th < 1)) {
            std::fclose(f);
            return fail(ctx, SDM_E_INVALID, "%s holds another render", path);
        }
        std::vector<uint8_t> done;
        std::vector<double> acc;
        if (ok) {
            done.resize((size_t)n_items);
            acc.resize(n_acc);
            ok = std::fread(done.data(), 1, done.size(), f) == done.size() &&
                 std::fread(acc.data(), sizeof(double), acc.size(), f) == acc.size();
        }
        std::fclose(f);
        if (!ok) return fail(ctx, SDM_E_INVALID, "%s is not a complete checkpoint", path);
        HIPCHK(ctx, hipSetDevice(ctx->device));
        HIPCHK(ctx, ctx->acc.ensure(n_acc * sizeof(double)));
        HIPCHK(ctx, hipMemcpy(ctx->acc.p, acc.data(), n_acc * sizeof(double), hipMemcpyHostToDevice));
        sdm_context::Partial &pt = ctx->partial;
        pt.valid = true;
        pt.digest = digest;
        pt.tw = tw;
        pt.th = th;
        pt.done.swap(done);
        pt.acc_elems = n_acc;
    } else if (!ctx->partial.valid || ctx->partial.digest != digest) {
        return fail(ctx, SDM_E_INVALID, "the context holds no partial render of these parameters");
    }
    Budget bud;
    bud.max_items = p->max_items;
    bud.resume = true;
    bud.digest = digest;
    return render_any(ctx, {j}, out->stats, (hipStream_t)hip_stream, bud);
}

int sdm_render_batch(sdm_context *ctx, int32_t n_jobs, const sdm_job *jobs, sdm_stats *stats, void *hip_stream)
{
    if (!ctx) return SDM_E_INVALID;
    if (n_jobs < 1 || !jobs) return fail(ctx, SDM_E_INVALID, "need at least one job");
    if (n_jobs >= (1 << (32 - kAuxJobShift))) return fail(ctx, SDM_E_UNSUPPORTED, "too many jobs");
    std::vector<JobIn> js;
    for (int32_t i = 0; i < n_jobs; ++i) {
        if (!jobs[i].params) return fail(ctx, SDM_E_INVALID, "job %d has no parameters", i);
        js.push_back({jobs[i].scene, jobs[i].params, jobs[i].out});
        if (int rc = check_job(ctx, js.back())) return rc;
        if (jobs[i].params->max_items > 0)
            return fail(ctx, SDM_E_UNSUPPORTED, "item budgets apply to single renders");
        if (jobs[i].scene->dev.dd.n_cells > 0)
            return fail(ctx, SDM_E_UNSUPPORTED, "scenes cut into sub-domains render singly");
        if (jobs[i].params->photons > 0)
            return fail(ctx, SDM_E_UNSUPPORTED, "the photon map applies to single renders");
    }
    ctx->partial.valid = false;
    // Scheduling: a job of at least half a chunk of paths fills the device on
    // its own and renders alone, through the one-job kernels (scene constants
    // uniform across the wave); smaller jobs, in their order, share
    // wavefronts of up to one chunk of paths, whose job table gives each path
    // its scene.  Every image is the same either way.
    const hipStream_t s = (hipStream_t)hip_stream;
    uint64_t chunk;
    int tw, th;
    job_shape(ctx, js[0], chunk, tw, th);
    sdm_stats total{};
    std::vector<JobIn> group;
    uint64_t gpaths = 0;
    auto run = [&](const std::vector<JobIn> &g) -> int {
        sdm_stats st{};
        if (int rc = render_any(ctx, g, &st, s)) return rc;
        add_stats(total, st);
        return SDM_OK;
    };
    for (const JobIn &j : js) {
        const uint64_t paths = (uint64_t)j.p->camera.W * j.p->camera.H * j.p->spp * j.p->n_bands;
        if (paths >= chunk / 2) {
            if (int rc = run({j})) return rc;
            continue;
        }
        if (!group.empty() && gpaths + paths > chunk) {
            if (int rc = run(group)) return rc;
            group.clear();
            gpaths = 0;
        }
        group.push_back(j);
        gpaths += paths;
    }
    if (!group.empty())
        if (int rc = run(group)) return rc;
    if (stats) *stats = total;
    return SDM_OK;
}

int sdm_autotune(sdm_context *ctx, const sdm_scene *sc, const sdm_render_params *p, const char *cache_path,
                 sdm_tune_result *res, void *hip_stream)
{
    if (!ctx) return SDM_E_INVALID;
    if (!sc || !p || !res) return fail(ctx, SDM_E_INVALID, "null argument");
    if (sc->ctx != ctx) return fail(ctx, SDM_E_INVALID, "scene belongs to another context");
    if (int rc = validate_params(ctx, p)) return rc;
    if (int rc = validate_btdf(ctx, sc, p)) return rc;
    std::memset(res, 0, sizeof(*res));
    const int W = p->camera.W, H = p->camera.H;
    char key[160];
    snprintf(key, sizeof(key), "nt=%d nmat=%d W=%d H=%d nl=%d depth=%d prec=%d bands=%d", sc->nt, sc->n_mat, W, H,
             p->n_lambda, p->max_depth, p->precision, p->n_bands);
    bool found = false;
    if (cache_path) {
        if (FILE *f = std::fopen(cache_path, "r")) {
            char line[256];
            while (std::fgets(line, sizeof(line), f)) {
                long long ch;
                int tw, th, tb, sb;
                double ms;
                const size_t kl = std::strlen(key);
                if (std::strncmp(line, key, kl) == 0 && line[kl] == ' ' &&
                    std::sscanf(line + kl, " -> chunk=%lld tile=%dx%d trace_bpc=%d shadow_bpc=%d ms=%lf", &ch, &tw,
                                &th, &tb, &sb, &ms) == 6) {
                    res->chunk_paths = ch;
                    res->tile_w = tw;
                    res->tile_h = th;
                    res->trace_blocks_per_cu = tb;
                    res->shadow_blocks_per_cu = sb;
                    res->ms = ms;
                    res->from_cache = 1;
                    found = true;
                }
            }
            std::fclose(f);
        }
    }
    if (!found) {
        // measure the render itself (a chunk size only matters relative to the
        // whole workload); outputs are not needed
        HIPCHK(ctx, hipSetDevice(ctx->device));
        sdm_render_params q = *p;
        q.timing = 0;
        q.graph = 0;
        q.max_items = 0;
        ctx->partial.valid = false;
        sdm_outputs none{};
        sdm_stats st{};
        none.stats = &st;
        auto time_it = [&](double &ms) -> int {
            ms = 1e300;
            for (int rep = 0; rep < 2; ++rep) {
                const JobIn j{sc, &q, &none};
                if (int rc = render_any(ctx, {j}, &st, (hipStream_t)hip_stream)) return rc;
                ms = std::min(ms, st.ms_render);
            }
            return SDM_OK;
        };
        // 1. chunk size and tile at the default blocks per CU
        const long long chunks[3] = {1ll << 22, 1ll << 23, 1ll << 24};
        const int tiles[3] = {8, 16, 32};
        double best = 1e300;
        const bool fp64 = p->precision == SDM_PREC_FP64;
        const int occ_t = fp64 ? occupancy<double>(SDM_K_TRACE) : occupancy<float>(SDM_K_TRACE);
        const int occ_s = fp64 ? occupancy<double>(SDM_K_SHADOW) : occupancy<float>(SDM_K_SHADOW);
        const int def_s = sc->dev.g_use ? std::min(4, occ_s) : occ_s;
        q.trace_blocks_per_cu = occ_t;
        q.shadow_blocks_per_cu = def_s;
        for (long long ch : chunks)
            for (int t : tiles) {
                q.chunk_paths = ch;
                q.tile_w = q.tile_h = t;
                double ms;
                if (int rc = time_it(ms)) return rc;
                if (ms < best) {
                    best = ms;
                    res->chunk_paths = ch;
                    res->tile_w = res->tile_h = t;
                }
            }
        q.chunk_paths = res->chunk_paths;
        q.tile_w = res->tile_w;
        q.tile_h = res->tile_h;
        // 2. resident blocks per CU of the closest-hit pass, then of the shadow
        // walk, from the most that fit down to half
        res->trace_blocks_per_cu = occ_t;
        for (int b = occ_t - 1; b >= std::max(1, (occ_t + 1) / 2); --b) {
            q.trace_blocks_per_cu = b;
            double ms;
            if (int rc = time_it(ms)) return rc;
            if (ms < best) {
                best = ms;
                res->trace_blocks_per_cu = b;
            }
        }
        q.trace_blocks_per_cu = res->trace_blocks_per_cu;
        res->shadow_blocks_per_cu = def_s;
        for (int b = occ_s; b >= std::max(1, (occ_s + 1) / 2); --b) {
            if (b == def_s) continue;
            q.shadow_blocks_per_cu = b;
            double ms;
            if (int rc = time_it(ms)) return rc;
            if (ms < best) {
                best = ms;
                res->shadow_blocks_per_cu = b;
            }
        }
        res->ms = best;
        if (cache_path)
            if (FILE *f = std::fopen(cache_path, "a")) {
                std::fprintf(f, "%s -> chunk=%lld tile=%dx%d trace_bpc=%d shadow_bpc=%d ms=%.4f\n", key,
                             (long long)res->chunk_paths, res->tile_w, res->tile_h, res->trace_blocks_per_cu,
                             res->shadow_blocks_per_cu, res->ms);
                std::fclose(f);
            }
    }
    auto &tv = ctx->tuned;
    tv.erase(std::remove_if(tv.begin(), tv.end(),
                            [&](const sdm_context::Tuned &t) {
                                return t.scene == sc && t.W == W && t.H == H && t.nl == p->n_lambda &&
                                       t.depth == p->max_depth && t.precision == p->precision;
                            }),
             tv.end());
    tv.push_back({sc, W, H, p->n_lambda, p->max_depth, p->precision, res->chunk_paths, res->tile_w, res->tile_h,
                  res->trace_blocks_per_cu, res->shadow_blocks_per_cu});
    return SDM_OK;
}

}  // extern "C"
