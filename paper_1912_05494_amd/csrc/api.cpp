// api.cpp -- C ABI of the spectral wavefront path tracer (see include/sdm.h).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <initializer_list>
#include <string>
#include <vector>

#include "../../include/sdm.h"
#include "bvh_build.hpp"
#include "subdomain.hpp"
#include "sun_grid.hpp"
#include "sdm_types.hpp"
#include "surrogate.hpp"
#include "wavefront.hpp"

using namespace sdm;

#include "runtime.hpp"

using namespace sdm_rt;

namespace sdm_rt {

int fail(sdm_context *ctx, int code, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    if (ctx) ctx->err = buf;
    return code;
}

bool ptr_is_device(const void *p)
{
    hipPointerAttribute_t a;
    if (hipPointerGetAttributes(&a, p) != hipSuccess) {
        (void)hipGetLastError();
        return false;
    }
    return a.type == hipMemoryTypeDevice;
}

}  // namespace sdm_rt

namespace {

int mlp_check(sdm_mlp *net, int64_t m, const void *tuples, const void *panes)
{
    if (m < 0 || m > (1LL << 30)) return fail(net->ctx, SDM_E_INVALID, "sample count %lld out of range", (long long)m);
    if (m > 0 && (!tuples || !panes)) return fail(net->ctx, SDM_E_INVALID, "null array");
    return SDM_OK;
}

int mlp_grad_blocks(const sdm_mlp *net, int64_t m)
{
    const int64_t waves = (m + 15) / 16;
    return (int)std::max<int64_t>(1, std::min<int64_t>(net->ctx->num_cu, (waves + 3) / 4));
}

// Enqueues pack + gradient + reduce for m samples; loss_dst receives the mean
// loss (device float).
int mlp_enqueue_grad(sdm_mlp *net, int64_t m, const float *tuples, const int32_t *panes, const float *target,
                     float *grad, float *loss_dst, hipStream_t s)
{
    sdm_context *ctx = net->ctx;
    const int nblk = mlp_grad_blocks(net, m);
    HIPCHK(ctx, net->partial.ensure((size_t)nblk * net->P * sizeof(float)));
    HIPCHK(ctx, net->loss_partial.ensure((size_t)nblk * sizeof(float)));
    launch_mlp_pack(net->params.as<float>(), net->wb.p, net->bb.as<float>(), s);
    launch_mlp_grad((uint32_t)m, net->n_panes, tuples, panes, target, net->wb.p, net->bb.as<float>(),
                    net->params.as<float>() + mlp_net_params(), 1.0f / (float)m, net->partial.as<float>(),
                    net->loss_partial.as<float>(), ctx->flag.as<int>(), nblk, s);
    launch_mlp_reduce(nblk, (int)net->P, net->partial.as<float>(), net->loss_partial.as<float>(), 1.0f / (float)m, grad,
                      loss_dst, s);
    return SDM_OK;
}

// Vertex p as (p[k + 1], p[k + 2], p[k]) (indices mod 3), w kept: the frame
// of the FP32 triangle test of rays whose dominant axis is k.
float4 rot_vertex(const float4 &p, int k)
{
    const float c[3] = {p.x, p.y, p.z};
    return make_float4(c[(k + 1) % 3], c[(k + 2) % 3], c[k], p.w);
}

// Copies k = ks[0], ks[1], ... of n triangles (TriDev or GridCand), one after
// the other.
template <class T>
std::vector<T> rotated_copies(const T *src, size_t n, std::initializer_list<int> ks)
{
    std::vector<T> out;
    out.reserve(n * ks.size());
    for (const int k : ks)
        for (size_t i = 0; i < n; ++i) {
            T t = src[i];
            t.a = rot_vertex(t.a, k);
            t.b = rot_vertex(t.b, k);
            t.c = rot_vertex(t.c, k);
            out.push_back(t);
        }
    return out;
}

// The dominant axis of a direction as the kernels' ray shear takes it.
int dominant_axis(const float d[3])
{
    const float ax = std::fabs(d[0]), ay = std::fabs(d[1]), az = std::fabs(d[2]);
    return (ax >= ay && ax >= az) ? 0 : (ay >= az ? 1 : 2);
}

int check_flag(sdm_context *ctx, hipStream_t s, const char *what)
{
    int bad = 0;
    HIPCHK(ctx, hipMemcpyAsync(&bad, ctx->flag.p, sizeof(int), hipMemcpyDeviceToHost, s));
    HIPCHK(ctx, hipStreamSynchronize(s));
    if (bad) return fail(ctx, SDM_E_INVALID, "%s: pane index out of range", what);
    return SDM_OK;
}

}  // namespace

extern "C" {

int sdm_context_create(int device, sdm_context **out)
{
    if (!out) return SDM_E_INVALID;
    *out = nullptr;
    int n = 0;
    if (hipGetDeviceCount(&n) != hipSuccess || device < 0 || device >= n) return SDM_E_DEVICE;
    if (hipSetDevice(device) != hipSuccess) return SDM_E_DEVICE;
    auto *ctx = new sdm_context();
    ctx->device = device;
    if (const char *fa = std::getenv("SDM_FAIL_ALLOC")) sdm_rt::fail_alloc_countdown().store(std::atol(fa));
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, device) != hipSuccess) {
        delete ctx;
        return SDM_E_DEVICE;
    }
    ctx->num_cu = prop.multiProcessorCount;
    // the allocation-free Monte Carlo entry point uses the device's static
    // scratch: resolve its address now, with the device current (on failure
    // that entry point reports an error; nothing else depends on it)
    if (mc_scratch_address(device, &ctx->mc_scratch) != 0) {
        ctx->mc_scratch = nullptr;
        (void)hipGetLastError();
    }
    if (hipHostMalloc((void **)&ctx->host_counters, sizeof(Counters), hipHostMallocDefault) != hipSuccess) {
        delete ctx;
        return SDM_E_NOMEM;
    }
    // the stream graphs are captured on and replayed from (default priority)
    if (hipStreamCreateWithFlags(&ctx->gstream, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&ctx->join[0], hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&ctx->join[1], hipEventDisableTiming) != hipSuccess ||
        hipStreamCreateWithFlags(&ctx->side, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&ctx->fork, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&ctx->rejoin, hipEventDisableTiming) != hipSuccess) {
        (void)sdm_context_destroy(ctx);
        return SDM_E_DEVICE;
    }
    if (const char *ser = std::getenv("SDM_SERIAL")) ctx->overlap = std::atoi(ser) == 0;
    *out = ctx;
    return SDM_OK;
}

int sdm_context_destroy(sdm_context *ctx)
{
    if (!ctx) return SDM_E_INVALID;
    (void)hipSetDevice(ctx->device);
    (void)hipDeviceSynchronize();
    for (auto e : ctx->events) (void)hipEventDestroy(e);
    if (ctx->gexec) (void)hipGraphExecDestroy(ctx->gexec);
    for (auto e : ctx->join)
        if (e) (void)hipEventDestroy(e);
    if (ctx->fork) (void)hipEventDestroy(ctx->fork);
    if (ctx->rejoin) (void)hipEventDestroy(ctx->rejoin);
    if (ctx->gstream) (void)hipStreamDestroy(ctx->gstream);
    if (ctx->side) (void)hipStreamDestroy(ctx->side);
    if (ctx->host_counters) (void)hipHostFree(ctx->host_counters);
    delete ctx;
    return SDM_OK;
}

const char *sdm_last_error(const sdm_context *ctx) { return ctx ? ctx->err.c_str() : "null context"; }

int sdm_scene_info(const sdm_scene *sc, int32_t *n_nodes, int32_t *depth, int32_t *stack, int64_t *grid_cells,
                   int64_t *grid_candidates)
{
    if (!sc) return SDM_E_INVALID;
    if (n_nodes) *n_nodes = sc->n_nodes;
    if (depth) *depth = sc->depth;
    if (stack) *stack = sc->stack;
    if (grid_cells) *grid_cells = sc->grid_cells;
    if (grid_candidates) *grid_candidates = sc->grid_cands;
    return SDM_OK;
}

int sdm_scene_create(sdm_context *ctx, const sdm_scene_desc *d, sdm_scene **out)
{
    if (!ctx) return SDM_E_INVALID;
    if (!d || !out) return fail(ctx, SDM_E_INVALID, "null scene description or output");
    *out = nullptr;
    if (d->nv < 0 || d->nt < 0) return fail(ctx, SDM_E_INVALID, "negative vertex/triangle count");
    if (d->shadow_walk != SDM_SHADOW_AUTO && d->shadow_walk != SDM_SHADOW_BVH)
        return fail(ctx, SDM_E_INVALID, "unknown shadow walk %d", d->shadow_walk);
    if (d->nt > 0 && (!d->pos || !d->idx || !d->mat || !d->mats || d->n_mat < 1))
        return fail(ctx, SDM_E_INVALID, "triangles need pos, idx, mat and materials");
    if (d->n_tab < 1 || !d->tab_lambda_nm || !d->sun_E || !d->sky_L)
        return fail(ctx, SDM_E_INVALID, "scene needs tab_lambda_nm, sun_E and sky_L tables");
    for (int i = 1; i < d->n_tab; ++i)
        if (!(d->tab_lambda_nm[i] > d->tab_lambda_nm[i - 1]))
            return fail(ctx, SDM_E_INVALID, "tab_lambda_nm must be strictly increasing");
    if ((int64_t)d->nt >= (int64_t)kMaxTris - 1) return fail(ctx, SDM_E_UNSUPPORTED, "too many triangles");
    for (int32_t t = 0; t < d->nt; ++t) {
        for (int c = 0; c < 3; ++c)
            if (d->idx[3 * (size_t)t + c] < 0 || d->idx[3 * (size_t)t + c] >= d->nv)
                return fail(ctx, SDM_E_INVALID, "triangle %d has a vertex index out of range", t);
        if (d->mat[t] < 0 || d->mat[t] >= d->n_mat)
            return fail(ctx, SDM_E_INVALID, "triangle %d has a material index out of range", t);
    }
    for (int32_t m = 0; m < d->n_mat; ++m) {
        const sdm_material &mm = d->mats[m];
        if (mm.type == SDM_LAMBERT) {
            if (!mm.albedo) return fail(ctx, SDM_E_INVALID, "Lambert material %d needs albedo", m);
        } else if (mm.type == SDM_GLASS || mm.type == SDM_GLASS_BUBBLY) {
            if (!mm.n || !mm.k) return fail(ctx, SDM_E_INVALID, "glass material %d needs n and k", m);
            for (int i = 0; i < d->n_tab; ++i)
                if (!(mm.n[i] >= 1.0f) || !(mm.k[i] >= 0.0f))
                    return fail(ctx, SDM_E_INVALID, "glass material %d needs n >= 1 and k >= 0", m);
            if (mm.type == SDM_GLASS_BUBBLY &&
                (!(mm.bubble_density_mm3 >= 0.0f) || !(mm.bubble_rmin_um >= 0.0f) ||
                 !(mm.bubble_rmax_um >= mm.bubble_rmin_um) || mm.pane_id < 0 || mm.pane_id >= kMaxPanes))
                return fail(ctx, SDM_E_INVALID,
                            "bubbly material %d needs density >= 0, 0 <= rmin <= rmax and pane_id in [0, %d)", m,
                            kMaxPanes);
        } else {
            return fail(ctx, SDM_E_INVALID, "material %d has an unknown type %d", m, mm.type);
        }
    }
    // distribution maps
    if (d->n_maps < 0 || (d->n_maps > 0 && !d->maps)) return fail(ctx, SDM_E_INVALID, "bad distribution map list");
    bool any_map = false;
    for (int32_t m = 0; m < d->n_mat; ++m) {
        const sdm_material &mm = d->mats[m];
        if (mm.dist_map == 0) continue;
        if (mm.type != SDM_GLASS)
            return fail(ctx, SDM_E_UNSUPPORTED, "material %d: distribution maps apply to clear glass only", m);
        if (mm.dist_map < 0 || mm.dist_map > d->n_maps)
            return fail(ctx, SDM_E_INVALID, "material %d names distribution map %d of %d", m, mm.dist_map - 1,
                        d->n_maps);
        any_map = true;
    }
    if (any_map && !d->uv) return fail(ctx, SDM_E_INVALID, "distribution maps need per-vertex uv");
    for (int32_t q = 0; q < d->n_maps; ++q) {
        const sdm_dist_map &dm = d->maps[q];
        if (dm.W < 1 || dm.H < 1 || dm.W > 4096 || dm.H > 4096 || !dm.material)
            return fail(ctx, SDM_E_INVALID, "distribution map %d needs 1 <= W, H <= 4096 and materials", q);
        for (int64_t x = 0; x < (int64_t)dm.W * dm.H; ++x) {
            const int32_t tm = dm.material[x];
            if (tm < 0 || tm >= d->n_mat || d->mats[tm].type != SDM_GLASS || d->mats[tm].dist_map != 0)
                return fail(ctx, SDM_E_INVALID,
                            "distribution map %d: texel %lld must name a clear-glass material without a map", q,
                            (long long)x);
            if (dm.thick_mm && !(dm.thick_mm[x] > 0.0f && dm.thick_mm[x] < 1e6f))
                return fail(ctx, SDM_E_INVALID, "distribution map %d: texel %lld thickness must be > 0", q,
                            (long long)x);
        }
    }
    if (d->uv)
        for (int64_t i = 0; i < 2 * (int64_t)d->nv; ++i)
            if (!std::isfinite(d->uv[i])) return fail(ctx, SDM_E_INVALID, "uv must be finite");
    int32_t dd_n[3];
    for (int a = 0; a < 3; ++a) {
        dd_n[a] = d->subdomains[a] < 1 ? 1 : d->subdomains[a];
        if (d->subdomains[a] < 0 || dd_n[a] > kMaxCellsPerAxis)
            return fail(ctx, SDM_E_INVALID, "subdomains must be in [0, %d] along each axis", kMaxCellsPerAxis);
    }
    if ((int64_t)dd_n[0] * dd_n[1] * dd_n[2] > 4096) return fail(ctx, SDM_E_INVALID, "at most 4096 sub-domains");
    const bool use_dd = (int64_t)dd_n[0] * dd_n[1] * dd_n[2] > 1 && d->nt > 0;
    if (d->subdomain_handoff != SDM_HANDOFF_QUEUE && d->subdomain_handoff != SDM_HANDOFF_MARCH)
        return fail(ctx, SDM_E_INVALID, "unknown sub-domain hand-off %d", d->subdomain_handoff);
    HIPCHK(ctx, hipSetDevice(ctx->device));
    auto *sc = new sdm_scene();
    sc->ctx = ctx;
    {
        // digest of every input that decides the rendered values (checkpoints)
        Digest dg;
        dg.add_value(d->nv);
        dg.add_value(d->nt);
        dg.add_value(d->n_mat);
        dg.add_value(d->n_tab);
        dg.add(d->pos, sizeof(float) * 3 * (size_t)d->nv);
        if (d->vthick_mm) dg.add(d->vthick_mm, sizeof(float) * (size_t)d->nv);
        dg.add(d->idx, sizeof(int32_t) * 3 * (size_t)d->nt);
        dg.add(d->mat, sizeof(int32_t) * (size_t)d->nt);
        dg.add(d->tab_lambda_nm, sizeof(float) * (size_t)d->n_tab);
        dg.add(d->sun_dir, sizeof(d->sun_dir));
        dg.add(d->sun_E, sizeof(float) * (size_t)d->n_tab);
        dg.add(d->sky_L, sizeof(float) * (size_t)d->n_tab);
        for (int32_t m = 0; m < d->n_mat; ++m) {
            const sdm_material &mm = d->mats[m];
            dg.add_value(mm.type);
            dg.add_value(mm.thick_mm);
            dg.add_value(mm.bubble_density_mm3);
            dg.add_value(mm.bubble_rmin_um);
            dg.add_value(mm.bubble_rmax_um);
            dg.add_value(mm.pane_id);
            for (const float *t : {mm.albedo, mm.n, mm.k, mm.alpha_tint})
                if (t) dg.add(t, sizeof(float) * (size_t)d->n_tab);
            dg.add_value(mm.dist_map);
        }
        if (d->uv) dg.add(d->uv, sizeof(float) * 2 * (size_t)d->nv);
        dg.add_value(d->n_maps);
        dg.add(d->subdomains, sizeof(d->subdomains));
        dg.add_value(d->subdomain_handoff);
        for (int32_t q = 0; q < d->n_maps; ++q) {
            const sdm_dist_map &dm = d->maps[q];
            dg.add_value(dm.W);
            dg.add_value(dm.H);
            dg.add(dm.material, sizeof(int32_t) * (size_t)dm.W * dm.H);
            if (dm.thick_mm) dg.add(dm.thick_mm, sizeof(float) * (size_t)dm.W * dm.H);
        }
        sc->digest = dg.h;
    }
    sc->n_tab = d->n_tab;
    sc->n_mat = d->n_mat;
    sc->nt = d->nt;
    BvhResult bvh = build_bvh(d->pos, d->nv, d->idx, d->nt);
    if (!bvh.ok) {
        delete sc;
        return fail(ctx, SDM_E_UNSUPPORTED, "scene too degenerate: a BVH leaf at the depth limit holds > %d triangles",
                    kMaxLeafTris);
    }
    sc->depth = bvh.depth;
    sc->stack = bvh.stack;
    sc->n_nodes = (int32_t)bvh.nodes.size();
    std::vector<TriDev> tris(d->nt);
    std::vector<float4> thick(d->nt);
    std::vector<int32_t> o2l(std::max(1, d->nt));
    for (int32_t l = 0; l < d->nt; ++l) {
        const int32_t t = bvh.order[l];
        o2l[t] = l;
        const float *p0 = d->pos + 3 * (size_t)d->idx[3 * (size_t)t];
        const float *p1 = d->pos + 3 * (size_t)d->idx[3 * (size_t)t + 1];
        const float *p2 = d->pos + 3 * (size_t)d->idx[3 * (size_t)t + 2];
        int32_t tt = t, mm = d->mat[t];
        float ft, fm;
        std::memcpy(&ft, &tt, 4);
        std::memcpy(&fm, &mm, 4);
        tris[l].a = make_float4(p0[0], p0[1], p0[2], ft);
        tris[l].b = make_float4(p1[0], p1[1], p1[2], fm);
        tris[l].c = make_float4(p2[0], p2[1], p2[2], 0.0f);   // w: material type, set below
        if (d->vthick_mm)
            thick[l] = make_float4(d->vthick_mm[d->idx[3 * (size_t)t]], d->vthick_mm[d->idx[3 * (size_t)t + 1]],
                                   d->vthick_mm[d->idx[3 * (size_t)t + 2]], 0.0f);
        else
            thick[l] = make_float4(0, 0, 0, 0);
    }
    // self-intersection epsilon: 1e-6 x diagonal of the vertex bounding box
    double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
    for (int32_t v = 0; v < d->nv; ++v)
        for (int a = 0; a < 3; ++a) {
            lo[a] = std::min(lo[a], (double)d->pos[3 * (size_t)v + a]);
            hi[a] = std::max(hi[a], (double)d->pos[3 * (size_t)v + a]);
        }
    double diag = 0.0;
    if (d->nv > 0)
        diag = std::sqrt((hi[0] - lo[0]) * (hi[0] - lo[0]) + (hi[1] - lo[1]) * (hi[1] - lo[1]) +
                         (hi[2] - lo[2]) * (hi[2] - lo[2]));
    std::vector<int32_t> mtype(d->n_mat);
    std::vector<float> mthick(d->n_mat);
    std::vector<float> tabm(4 * (size_t)d->n_mat * d->n_tab, 0.0f);
    std::vector<double> mbub(4 * (size_t)std::max(1, d->n_mat), 0.0);
    for (int32_t m = 0; m < d->n_mat; ++m) {
        const sdm_material &mm = d->mats[m];
        mtype[m] = mm.type == SDM_LAMBERT ? 0 : (mm.type == SDM_GLASS ? 1 : 2);
        if (mm.type == SDM_LAMBERT) {
            // a flat albedo table is gray: its bounces scale every wavelength alike
            bool flat = true;
            for (int i = 1; i < d->n_tab; ++i) flat = flat && mm.albedo[i] == mm.albedo[0];
            if (flat) mtype[m] = 3;
        }
        mthick[m] = mm.thick_mm;
        if (mm.type == SDM_GLASS_BUBBLY) {
            // extinction rho_b pi <r^2> (r ~ U(rmin, rmax), mm) and the inner index:
            // the material's n at kLambdaRef, interpolated linearly in its table
            const double a = (double)mm.bubble_rmin_um * 1e-3, b = (double)mm.bubble_rmax_um * 1e-3;
            mbub[4 * (size_t)m] = (double)mm.bubble_density_mm3 * M_PI * ((a * a + a * b + b * b) / 3.0);
            const double x = kLambdaRef;
            const float *tx = d->tab_lambda_nm, *ty = mm.n;
            double nref;
            if (d->n_tab == 1 || x <= tx[0]) {
                nref = ty[0];
            } else if (x >= tx[d->n_tab - 1]) {
                nref = ty[d->n_tab - 1];
            } else {
                int i = 0;
                while ((double)tx[i + 1] < x) ++i;
                const double wgt = (x - tx[i]) / ((double)tx[i + 1] - tx[i]);
                nref = (1.0 - wgt) * ty[i] + wgt * ty[i + 1];
            }
            mbub[4 * (size_t)m + 1] = nref;
            mbub[4 * (size_t)m + 2] = mm.bubble_density_mm3;
            mbub[4 * (size_t)m + 3] = mm.pane_id;
            sc->max_pane = std::max(sc->max_pane, mm.pane_id);
        }
        const float *src[4] = {mm.albedo, mm.n, mm.k, mm.alpha_tint};
        for (int q = 0; q < 4; ++q)
            if (src[q])
                std::memcpy(&tabm[((size_t)q * d->n_mat + m) * d->n_tab], src[q], sizeof(float) * d->n_tab);
    }
    // each triangle carries its material type in c.w, read with its vertices
    for (int32_t l = 0; l < d->nt; ++l) {
        int32_t m;
        std::memcpy(&m, &tris[l].b.w, 4);
        const int32_t ty = mtype[m];
        std::memcpy(&tris[l].c.w, &ty, 4);
    }
    // bounds of the triangles (vertices no triangle uses do not count): the
    // region the BVH padding and the sub-domain grid are sized for
    double tlo[3] = {INFINITY, INFINITY, INFINITY}, thi[3] = {-INFINITY, -INFINITY, -INFINITY};
    for (int64_t i = 0; i < 3 * (int64_t)d->nt; ++i)
        for (int a = 0; a < 3; ++a) {
            tlo[a] = std::min(tlo[a], (double)d->pos[3 * (size_t)d->idx[i] + a]);
            thi[a] = std::max(thi[a], (double)d->pos[3 * (size_t)d->idx[i] + a]);
        }
    for (int a = 0; a < 3; ++a) {
        sc->lo[a] = d->nt > 0 ? tlo[a] : 0.0;
        sc->hi[a] = d->nt > 0 ? thi[a] : 0.0;
    }
    double maxabs = 0.0;
    for (int a = 0; a < 3 && d->nv > 0; ++a) maxabs = std::max({maxabs, std::fabs(lo[a]), std::fabs(hi[a])});
    const SunGrid grid = d->shadow_walk == SDM_SHADOW_BVH
                             ? SunGrid()
                             : build_sun_grid(tris.data(), d->nt, mtype.data(), d->sun_dir, diag + maxabs);
    hipError_t e = hipSuccess;
    auto chk = [&](hipError_t x) { if (e == hipSuccess) e = x; };
    const int sun_axis = dominant_axis(d->sun_dir);
    if (grid.use) {
        chk(upload(sc->g_start, grid.start.data(), grid.start.size()));
        chk(upload(sc->g_cand, grid.cand.data(), grid.cand.size()));
        const std::vector<GridCand> rc = rotated_copies(grid.cand.data(), grid.cand.size(), {sun_axis});
        chk(upload(sc->g_cand_rot, rc.data(), rc.size()));
    }
    chk(upload(sc->nodes, bvh.nodes.data(), bvh.nodes.size()));
    chk(upload(sc->tris, tris.data(), tris.size()));
    {
        const std::vector<TriDev> rt = rotated_copies(tris.data(), tris.size(), {0, 1, 2});
        chk(upload(sc->tris_rot, rt.data(), rt.size()));
    }
    chk(upload(sc->thick, thick.data(), thick.size()));
    chk(upload(sc->orig_to_leaf, o2l.data(), o2l.size()));
    chk(upload(sc->mat_type, mtype.data(), mtype.size()));
    chk(upload(sc->mat_thick, mthick.data(), mthick.size()));
    chk(upload(sc->mat_bub, mbub.data(), mbub.size()));
    if (any_map) {
        std::vector<int32_t> mmap(d->n_mat);
        for (int32_t m = 0; m < d->n_mat; ++m) mmap[m] = d->mats[m].dist_map - 1;
        std::vector<int4> hdr(d->n_maps);
        std::vector<int32_t> tmat;
        std::vector<float> tthick;
        for (int32_t q = 0; q < d->n_maps; ++q) {
            const sdm_dist_map &dm = d->maps[q];
            const size_t n = (size_t)dm.W * dm.H;
            hdr[q] = make_int4(dm.W, dm.H, (int)tmat.size(), dm.thick_mm ? 1 : 0);
            tmat.insert(tmat.end(), dm.material, dm.material + n);
            if (dm.thick_mm) tthick.insert(tthick.end(), dm.thick_mm, dm.thick_mm + n);
            else tthick.insert(tthick.end(), n, 0.0f);
        }
        std::vector<float4> tuv(2 * (size_t)d->nt);
        for (int32_t l = 0; l < d->nt; ++l) {
            const int32_t t = bvh.order[l];
            const float *q0 = d->uv + 2 * (size_t)d->idx[3 * (size_t)t];
            const float *q1 = d->uv + 2 * (size_t)d->idx[3 * (size_t)t + 1];
            const float *q2 = d->uv + 2 * (size_t)d->idx[3 * (size_t)t + 2];
            tuv[2 * (size_t)l] = make_float4(q0[0], q0[1], q1[0], q1[1]);
            tuv[2 * (size_t)l + 1] = make_float4(q2[0], q2[1], 0.0f, 0.0f);
        }
        chk(upload(sc->mat_map, mmap.data(), mmap.size()));
        chk(upload(sc->map_hdr, hdr.data(), hdr.size()));
        chk(upload(sc->map_mat, tmat.data(), tmat.size()));
        chk(upload(sc->map_thick, tthick.data(), tthick.size()));
        chk(upload(sc->tri_uv, tuv.data(), tuv.size()));
    }
    SubdomainBuild sub;
    if (use_dd) {
        sub = build_subdomains(d->pos, d->nv, d->idx, d->nt, tris, o2l, dd_n, sc->lo, sc->hi);
        if (!sub.ok) {
            delete sc;
            return fail(ctx, SDM_E_UNSUPPORTED, "a sub-domain's BVH has a leaf at the depth limit holding > %d triangles",
                        kMaxLeafTris);
        }
        chk(upload(sc->dd_cells, sub.cells.data(), sub.cells.size()));
        chk(upload(sc->dd_nodes, sub.nodes.data(), std::max<size_t>(1, sub.nodes.size())));
        chk(upload(sc->dd_tris, sub.tris.data(), std::max<size_t>(1, sub.tris.size())));
        chk(upload(sc->dd_leaf, sub.leaf.data(), std::max<size_t>(1, sub.leaf.size())));
        for (int a = 0; a < 3; ++a) sc->dd_n[a] = dd_n[a];
        sc->dd_refs = (int64_t)sub.tris.size();
        sc->dd_nodes_n = (int64_t)sub.nodes.size();
        sc->dd_stack = sub.stack;
    }
    chk(upload(sc->tab_x, d->tab_lambda_nm, (size_t)d->n_tab));
    chk(upload(sc->tab_mat, tabm.data(), tabm.size()));
    chk(upload(sc->tab_sun, d->sun_E, (size_t)d->n_tab));
    chk(upload(sc->tab_sky, d->sky_L, (size_t)d->n_tab));
    if (e == hipSuccess) e = hipDeviceSynchronize();
    if (e != hipSuccess) {
        delete sc;
        return fail(ctx, e == hipErrorOutOfMemory ? SDM_E_NOMEM : SDM_E_DEVICE, "scene upload: %s",
                    hipGetErrorString(e));
    }
    SceneDev &sd = sc->dev;
    sd.nodes = sc->nodes.as<BvhNode>();
    sd.tris = sc->tris.as<TriDev>();
    sd.tris_rot = sc->tris_rot.as<TriDev>();
    sd.rot_n = d->nt;
    sd.thick = sc->thick.as<float4>();
    sd.mat_type = sc->mat_type.as<int32_t>();
    sd.mat_thick = sc->mat_thick.as<float>();
    sd.mat_bub = sc->mat_bub.as<double>();
    sd.n_nodes = sc->n_nodes;
    sd.nt = d->nt;
    sd.n_mat = d->n_mat;
    sd.has_vthick = d->vthick_mm ? 1 : 0;
    for (int a = 0; a < 3; ++a) sd.sun[a] = d->sun_dir[a];
    sd.g_use = grid.use ? 1 : 0;
    sd.g_start = grid.use ? sc->g_start.as<int32_t>() : nullptr;
    sd.g_cand = grid.use ? sc->g_cand.as<GridCand>() : nullptr;
    sd.g_cand_rot = grid.use ? sc->g_cand_rot.as<GridCand>() : nullptr;
    sd.g_rot = sun_axis;
    for (int a = 0; a < 3; ++a) {
        sd.g_e1[a] = grid.e1[a];
        sd.g_e2[a] = grid.e2[a];
    }
    sd.g_u0 = grid.u0;
    sd.g_v0 = grid.v0;
    sd.g_idu = grid.idu;
    sd.g_idv = grid.idv;
    sd.g_marg = grid.marg;
    sd.g_nx = grid.nx;
    sd.g_ny = grid.ny;
    sc->grid_cells = (int64_t)grid.nx * grid.ny;
    sc->grid_cands = (int64_t)grid.cand.size();
    sd.teps_d = 1e-6 * diag;
    sd.teps_f = (float)sd.teps_d;
    sd.dd = DdDev{};
    if (use_dd) {
        for (int a = 0; a < 3; ++a) {
            sd.dd.n[a] = dd_n[a];
            sd.dd.lo[a] = sub.lo[a];
            sd.dd.size[a] = sub.size[a];
        }
        sd.dd.n_cells = dd_n[0] * dd_n[1] * dd_n[2];
        sd.dd.sweeps = (dd_n[0] + dd_n[1] + dd_n[2] + 2) / 3 * 3;
        sd.dd.march = d->subdomain_handoff == SDM_HANDOFF_MARCH ? 1 : 0;
        sd.dd.cells = sc->dd_cells.as<CellDev>();
        sd.dd.nodes = sc->dd_nodes.as<BvhNode>();
        sd.dd.tris = sc->dd_tris.as<TriDev>();
        sd.dd.leaf = sc->dd_leaf.as<int32_t>();
    }
    sd.n_maps = any_map ? d->n_maps : 0;
    sd.mat_map = any_map ? sc->mat_map.as<int32_t>() : nullptr;
    sd.map_hdr = any_map ? sc->map_hdr.as<int4>() : nullptr;
    sd.map_mat = any_map ? sc->map_mat.as<int32_t>() : nullptr;
    sd.map_thick = any_map ? sc->map_thick.as<float>() : nullptr;
    sd.tri_uv = any_map ? sc->tri_uv.as<float4>() : nullptr;
    *out = sc;
    return SDM_OK;
}

int sdm_scene_subdomains(const sdm_scene *sc, int32_t cells[3], int64_t *tri_refs, int64_t *nodes)
{
    if (!sc) return SDM_E_INVALID;
    if (cells)
        for (int a = 0; a < 3; ++a) cells[a] = sc->dd_n[a];
    if (tri_refs) *tri_refs = sc->dd_refs;
    if (nodes) *nodes = sc->dd_nodes_n;
    return SDM_OK;
}

int sdm_scene_destroy(sdm_scene *sc)
{
    if (!sc) return SDM_E_INVALID;
    (void)hipSetDevice(sc->ctx->device);
    (void)hipDeviceSynchronize();
    delete sc;
    return SDM_OK;
}

}  // extern "C"

extern "C" {

int sdm_slab_eval(sdm_context *ctx, int64_t m, const float *cos_i, const float *lambda_nm, const float *d_mm,
                  const float *n, const float *k, const float *alpha_tint, float *R, float *T, void *hip_stream)
{
    if (!ctx) return SDM_E_INVALID;
    if (m < 0) return fail(ctx, SDM_E_INVALID, "negative size");
    if (m == 0) return SDM_OK;
    if (!cos_i || !lambda_nm || !d_mm || !n || !k || !R || !T)
        return fail(ctx, SDM_E_INVALID, "null array");
    HIPCHK(ctx, hipSetDevice(ctx->device));
    launch_slab_eval(m, cos_i, lambda_nm, d_mm, n, k, alpha_tint, R, T, (hipStream_t)hip_stream);
    HIPCHK(ctx, hipGetLastError());
    return SDM_OK;
}

int sdm_debug_intersect(sdm_context *ctx, const sdm_scene *sc, int64_t m, const float *o, const float *d,
                        const int32_t *skip, float *t, int32_t *tri, float *uv, void *hip_stream)
{
    if (!ctx) return SDM_E_INVALID;
    if (!sc || m < 0 || m >= (1ll << 31)) return fail(ctx, SDM_E_INVALID, "bad scene or size");
    if (m == 0) return SDM_OK;
    if (!o || !d || !t || !tri || !uv) return fail(ctx, SDM_E_INVALID, "null array");
    HIPCHK(ctx, hipSetDevice(ctx->device));
    hipStream_t s = (hipStream_t)hip_stream;
    const int grid = (int)std::max<int64_t>(1, std::min<int64_t>(4LL * ctx->num_cu, (m + 255) / 256));
    HIPCHK(ctx, ctx->gstack.ensure((size_t)grid * block_size() * global_stack_levels(sc->stack) * sizeof(int32_t)));
    launch_debug_intersect(sc->dev, (uint32_t)m, o, d, skip, sc->orig_to_leaf.as<int32_t>(), t, tri, uv,
                           ctx->gstack.as<int32_t>(), grid, s);
    HIPCHK(ctx, hipGetLastError());
    return SDM_OK;
}

int sdm_debug_shadow(sdm_context *ctx, const sdm_scene *sc, int64_t m, const float *o, const int32_t *skip,
                     float lambda_nm, float *T, void *hip_stream)
{
    if (!ctx) return SDM_E_INVALID;
    if (!sc || m < 0 || m >= (1ll << 31)) return fail(ctx, SDM_E_INVALID, "bad scene or size");
    if (m == 0) return SDM_OK;
    if (!o || !T) return fail(ctx, SDM_E_INVALID, "null array");
    HIPCHK(ctx, hipSetDevice(ctx->device));
    hipStream_t s = (hipStream_t)hip_stream;
    const int nm = sc->n_mat;
    HIPCHK(ctx, ctx->slab_tmp.ensure(256 + 4 * (size_t)nm * sizeof(float)));
    float *lam = ctx->slab_tmp.as<float>();
    float *tabs = lam + 64;  // [4][nm] : rho, n, k, tint at lambda
    HIPCHK(ctx, hipMemcpyAsync(lam, &lambda_nm, sizeof(float), hipMemcpyHostToDevice, s));
    launch_resample<float>(sc->tab_x.as<float>(), sc->n_tab, sc->tab_mat.as<float>(), 4 * nm, lam, 1, 1, tabs, s);
    const int grid = (int)std::max<int64_t>(1, std::min<int64_t>(4LL * ctx->num_cu, (m + 255) / 256));
    HIPCHK(ctx, ctx->gstack.ensure((size_t)grid * block_size() * global_stack_levels(sc->stack) * sizeof(int32_t)));
    launch_debug_shadow(sc->dev, (uint32_t)m, o, skip, sc->orig_to_leaf.as<int32_t>(), lambda_nm, tabs + nm,
                        tabs + 2 * nm, tabs + 3 * nm, T,
                        ctx->gstack.as<int32_t>(), grid, s);
    HIPCHK(ctx, hipGetLastError());
    HIPCHK(ctx, hipStreamSynchronize(s));
    return SDM_OK;
}

int sdm_slab_mc(sdm_context *ctx, int64_t m, const float *cos_i, const float *lambda_nm, const float *d_mm,
                const float *rho_b, const float *n, const float *k, const float *alpha_tint, const float *n_ref,
                float rmin_um, float rmax_um, int32_t n_photons, uint64_t seed, uint32_t tuple0, int32_t precision,
                float *R, float *T, float *A, float *w_lobe, void *hip_stream)
{
    if (!ctx) return SDM_E_INVALID;
    if (m < 0 || m > 0xffffffffLL) return fail(ctx, SDM_E_INVALID, "tuple count %lld out of range", (long long)m);
    if (n_photons < 1) return fail(ctx, SDM_E_INVALID, "n_photons must be >= 1");
    if ((uint64_t)tuple0 + (uint64_t)m > 0x100000000ULL)
        return fail(ctx, SDM_E_INVALID, "tuple0 + m exceeds the 32-bit counter word");
    if (!(rmin_um >= 0.0f) || !(rmax_um >= rmin_um)) return fail(ctx, SDM_E_INVALID, "bad bubble radius range");
    if (precision != SDM_PREC_FP32 && precision != SDM_PREC_FP64) return fail(ctx, SDM_E_INVALID, "bad precision");
    if (m == 0) return SDM_OK;
    if (!cos_i || !lambda_nm || !d_mm || !rho_b || !n || !k || !R || !T || !w_lobe)
        return fail(ctx, SDM_E_INVALID, "null array");
    HIPCHK(ctx, hipSetDevice(ctx->device));
    hipStream_t s = (hipStream_t)hip_stream;
    HIPCHK(ctx, ctx->mc_acc.ensure(4 * (size_t)m * sizeof(double)));
    const double a = (double)rmin_um * 1e-3, b = (double)rmax_um * 1e-3;
    const double r2 = (a * a + a * b + b * b) / 3.0;   // <r^2> in mm^2, r ~ U(a, b)
    if (precision == SDM_PREC_FP64)
        launch_slab_mc<double>((uint32_t)m, (uint32_t)n_photons, cos_i, lambda_nm, d_mm, rho_b, n, k, alpha_tint,
                               n_ref, r2, seed, tuple0, ctx->mc_acc.as<double>(), R, T, A, w_lobe, ctx->num_cu, s);
    else
        launch_slab_mc<float>((uint32_t)m, (uint32_t)n_photons, cos_i, lambda_nm, d_mm, rho_b, n, k, alpha_tint,
                              n_ref, r2, seed, tuple0, ctx->mc_acc.as<double>(), R, T, A, w_lobe, ctx->num_cu, s);
    HIPCHK(ctx, hipGetLastError());
    HIPCHK(ctx, hipStreamSynchronize(s));
    return SDM_OK;
}

int sdm_slab_mc_noalloc(sdm_context *ctx, int64_t m, const float *cos_i, const float *lambda_nm, const float *d_mm,
                        const float *rho_b, const float *n, const float *k, const float *alpha_tint,
                        const float *n_ref, float rmin_um, float rmax_um, int32_t n_photons, uint64_t seed,
                        uint32_t tuple0, int32_t precision, float *R, float *T, float *A, float *w_lobe,
                        void *hip_stream)
{
    if (!ctx) return SDM_E_INVALID;
    if (m < 0 || m > (int64_t)kMcScratchTuples)
        return fail(ctx, SDM_E_INVALID, "tuple count %lld out of range [0, %u] (the static scratch holds %u tuples)",
                    (long long)m, kMcScratchTuples, kMcScratchTuples);
    if (n_photons < 1) return fail(ctx, SDM_E_INVALID, "n_photons must be >= 1");
    if ((uint64_t)tuple0 + (uint64_t)m > 0x100000000ULL)
        return fail(ctx, SDM_E_INVALID, "tuple0 + m exceeds the 32-bit counter word");
    if (!(rmin_um >= 0.0f) || !(rmax_um >= rmin_um)) return fail(ctx, SDM_E_INVALID, "bad bubble radius range");
    if (precision != SDM_PREC_FP32 && precision != SDM_PREC_FP64) return fail(ctx, SDM_E_INVALID, "bad precision");
    if (m == 0) return SDM_OK;
    if (!cos_i || !lambda_nm || !d_mm || !rho_b || !n || !k || !R || !T || !w_lobe)
        return fail(ctx, SDM_E_INVALID, "null array");
    if (!ctx->mc_scratch) return fail(ctx, SDM_E_DEVICE, "no static scratch on device %d", ctx->device);
    HIPCHK(ctx, hipSetDevice(ctx->device));
    hipStream_t s = (hipStream_t)hip_stream;
    const double a = (double)rmin_um * 1e-3, b = (double)rmax_um * 1e-3;
    const double r2 = (a * a + a * b + b * b) / 3.0;   // <r^2> in mm^2, r ~ U(a, b)
    // the scratch sums start from zero: launch_slab_mc clears them with a kernel
    if (precision == SDM_PREC_FP64)
        launch_slab_mc<double>((uint32_t)m, (uint32_t)n_photons, cos_i, lambda_nm, d_mm, rho_b, n, k, alpha_tint,
                               n_ref, r2, seed, tuple0, ctx->mc_scratch, R, T, A, w_lobe, ctx->num_cu, s);
    else
        launch_slab_mc<float>((uint32_t)m, (uint32_t)n_photons, cos_i, lambda_nm, d_mm, rho_b, n, k, alpha_tint,
                              n_ref, r2, seed, tuple0, ctx->mc_scratch, R, T, A, w_lobe, ctx->num_cu, s);
    HIPCHK(ctx, hipGetLastError());
    return SDM_OK;
}

int64_t sdm_mlp_nparams(int32_t n_panes) { return n_panes < 0 ? -1 : (int64_t)mlp_net_params() + 8LL * n_panes; }

int sdm_mlp_create(sdm_context *ctx, int32_t n_panes, const float *params, sdm_mlp **out)
{
    if (!ctx) return SDM_E_INVALID;
    if (!out || !params) return fail(ctx, SDM_E_INVALID, "null argument");
    *out = nullptr;
    if (n_panes < 1 || n_panes > kMaxPanes)
        return fail(ctx, SDM_E_INVALID, "n_panes must be in [1, %d]", kMaxPanes);
    HIPCHK(ctx, hipSetDevice(ctx->device));
    sdm_mlp *net = new sdm_mlp;
    net->ctx = ctx;
    net->n_panes = n_panes;
    net->P = sdm_mlp_nparams(n_panes);
    const size_t pb = (size_t)net->P * sizeof(float);
    hipError_t e = upload(net->params, params, (size_t)net->P);
    if (e == hipSuccess) e = net->m1.ensure(pb);
    if (e == hipSuccess) e = net->m2.ensure(pb);
    if (e == hipSuccess) e = net->wb.ensure((size_t)mlp_wb_elems() * 2);
    if (e == hipSuccess) e = net->bb.ensure((size_t)mlp_bb_elems() * sizeof(float));
    if (e == hipSuccess) e = hipMemset(net->m1.p, 0, pb);
    if (e == hipSuccess) e = hipMemset(net->m2.p, 0, pb);
    if (e == hipSuccess) e = hipDeviceSynchronize();
    if (e != hipSuccess) {
        delete net;
        return fail(ctx, e == hipErrorOutOfMemory ? SDM_E_NOMEM : SDM_E_DEVICE, "mlp create: %s",
                    hipGetErrorString(e));
    }
    *out = net;
    return SDM_OK;
}

int sdm_mlp_destroy(sdm_mlp *net)
{
    if (!net) return SDM_E_INVALID;
    (void)hipSetDevice(net->ctx->device);
    delete net;
    return SDM_OK;
}

int sdm_mlp_get_params(const sdm_mlp *net, float *params)
{
    if (!net) return SDM_E_INVALID;
    if (!params) return fail(net->ctx, SDM_E_INVALID, "null params");
    HIPCHK(net->ctx, hipSetDevice(net->ctx->device));
    HIPCHK(net->ctx, hipMemcpy(params, net->params.p, (size_t)net->P * sizeof(float), hipMemcpyDeviceToHost));
    return SDM_OK;
}


static const char kMlpMagic[8] = {'S', 'D', 'M', 'M', 'L', 'P', '0', '1'};

int sdm_mlp_save(const sdm_mlp *net, const char *path)
{
    if (!net) return SDM_E_INVALID;
    if (!path) return fail(net->ctx, SDM_E_INVALID, "null path");
    HIPCHK(net->ctx, hipSetDevice(net->ctx->device));
    const size_t P = (size_t)net->P;
    std::vector<float> buf(3 * P);
    HIPCHK(net->ctx, hipMemcpy(buf.data(), net->params.p, P * sizeof(float), hipMemcpyDeviceToHost));
    HIPCHK(net->ctx, hipMemcpy(buf.data() + P, net->m1.p, P * sizeof(float), hipMemcpyDeviceToHost));
    HIPCHK(net->ctx, hipMemcpy(buf.data() + 2 * P, net->m2.p, P * sizeof(float), hipMemcpyDeviceToHost));
    FILE *f = std::fopen(path, "wb");
    if (!f) return fail(net->ctx, SDM_E_DEVICE, "cannot open %s for writing", path);
    const int64_t np = net->P, t = net->t;
    bool ok = std::fwrite(kMlpMagic, 1, 8, f) == 8 && std::fwrite(&net->n_panes, 4, 1, f) == 1 &&
              std::fwrite(&np, 8, 1, f) == 1 && std::fwrite(&t, 8, 1, f) == 1 &&
              std::fwrite(buf.data(), sizeof(float), buf.size(), f) == buf.size();
    ok = (std::fclose(f) == 0) && ok;
    if (!ok) return fail(net->ctx, SDM_E_DEVICE, "write error on %s", path);
    return SDM_OK;
}

int sdm_mlp_load(sdm_context *ctx, const char *path, sdm_mlp **out)
{
    if (!ctx) return SDM_E_INVALID;
    if (!path || !out) return fail(ctx, SDM_E_INVALID, "null argument");
    *out = nullptr;
    FILE *f = std::fopen(path, "rb");
    if (!f) return fail(ctx, SDM_E_INVALID, "cannot open %s", path);
    char magic[8];
    int32_t n_panes = 0;
    int64_t np = 0, t = 0;
    bool ok = std::fread(magic, 1, 8, f) == 8 && std::memcmp(magic, kMlpMagic, 8) == 0 &&
              std::fread(&n_panes, 4, 1, f) == 1 && std::fread(&np, 8, 1, f) == 1 && std::fread(&t, 8, 1, f) == 1 &&
              n_panes >= 1 && n_panes <= kMaxPanes && np == sdm_mlp_nparams(n_panes) && t >= 0;
    std::vector<float> buf;
    if (ok) {
        buf.resize(3 * (size_t)np);
        ok = std::fread(buf.data(), sizeof(float), buf.size(), f) == buf.size();
    }
    std::fclose(f);
    if (!ok) return fail(ctx, SDM_E_INVALID, "%s is not a saved network", path);
    sdm_mlp *net = nullptr;
    if (int rc = sdm_mlp_create(ctx, n_panes, buf.data(), &net)) return rc;
    const size_t pb = (size_t)np * sizeof(float);
    hipError_t e = hipMemcpy(net->m1.p, buf.data() + np, pb, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(net->m2.p, buf.data() + 2 * np, pb, hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        sdm_mlp_destroy(net);
        return fail(ctx, e == hipErrorOutOfMemory ? SDM_E_NOMEM : SDM_E_DEVICE, "mlp load: %s",
                    hipGetErrorString(e));
    }
    net->t = t;
    *out = net;
    return SDM_OK;
}

int sdm_mlp_info(const sdm_mlp *net, int32_t *n_panes, int64_t *steps)
{
    if (!net) return SDM_E_INVALID;
    if (n_panes) *n_panes = net->n_panes;
    if (steps) *steps = net->t;
    return SDM_OK;
}

int sdm_mlp_grad(sdm_mlp *net, int64_t m, const float *tuples, const int32_t *panes, const float *target,
                 float *grad, float *loss, void *hip_stream)
{
    if (!net) return SDM_E_INVALID;
    sdm_context *ctx = net->ctx;
    if (int rc = mlp_check(net, m, tuples, panes)) return rc;
    if (m == 0) return fail(ctx, SDM_E_INVALID, "empty batch");
    if (!target || !grad) return fail(ctx, SDM_E_INVALID, "null array");
    HIPCHK(ctx, hipSetDevice(ctx->device));
    hipStream_t s = (hipStream_t)hip_stream;
    HIPCHK(ctx, ctx->flag.ensure(sizeof(int)));
    HIPCHK(ctx, net->loss.ensure(sizeof(float)));
    launch_zero_i32(ctx->flag.as<int>(), 1, s);
    if (int rc = mlp_enqueue_grad(net, m, tuples, panes, target, grad, net->loss.as<float>(), s)) return rc;
    HIPCHK(ctx, hipGetLastError());
    if (int rc = check_flag(ctx, s, "sdm_mlp_grad")) return rc;
    if (loss) HIPCHK(ctx, hipMemcpy(loss, net->loss.p, sizeof(float), hipMemcpyDeviceToHost));
    return SDM_OK;
}

int sdm_mlp_train(sdm_mlp *net, int64_t m, const float *tuples, const int32_t *panes, const float *target,
                  const sdm_train_params *tp, float *loss_curve, void *hip_stream)
{
    if (!net) return SDM_E_INVALID;
    sdm_context *ctx = net->ctx;
    if (int rc = mlp_check(net, m, tuples, panes)) return rc;
    if (!tp || !target) return fail(ctx, SDM_E_INVALID, "null argument");
    if (tp->steps < 0 || tp->batch < 1 || tp->batch > m)
        return fail(ctx, SDM_E_INVALID, "need 0 <= steps and 1 <= batch <= m");
    if (!(tp->lr > 0.0f) || !(tp->beta1 >= 0.0f && tp->beta1 < 1.0f) || !(tp->beta2 >= 0.0f && tp->beta2 < 1.0f) ||
        !(tp->eps > 0.0f))
        return fail(ctx, SDM_E_INVALID, "bad optimiser constants");
    if (tp->steps == 0) return SDM_OK;
    HIPCHK(ctx, hipSetDevice(ctx->device));
    hipStream_t s = (hipStream_t)hip_stream;
    HIPCHK(ctx, ctx->flag.ensure(sizeof(int)));
    HIPCHK(ctx, net->loss.ensure((size_t)tp->steps * sizeof(float)));
    launch_zero_i32(ctx->flag.as<int>(), 1, s);
    const int64_t nb = m / tp->batch;
    // two launches per step: the gradient pass (block rows) and the fused sum,
    // Adam step and repacking of the weights the next pass reads
    const int nblk = mlp_grad_blocks(net, tp->batch);
    HIPCHK(ctx, net->partial.ensure((size_t)nblk * net->P * sizeof(float)));
    HIPCHK(ctx, net->loss_partial.ensure((size_t)nblk * sizeof(float)));
    launch_mlp_pack(net->params.as<float>(), net->wb.p, net->bb.as<float>(), s);
    const float inv_n = 1.0f / (float)tp->batch;
    for (int32_t step = 0; step < tp->steps; ++step) {
        const int64_t off = (step % nb) * (int64_t)tp->batch;
        launch_mlp_grad((uint32_t)tp->batch, net->n_panes, tuples + 4 * off, panes + off, target + 3 * off, net->wb.p,
                        net->bb.as<float>(), net->params.as<float>() + mlp_net_params(), inv_n,
                        net->partial.as<float>(), net->loss_partial.as<float>(), ctx->flag.as<int>(), nblk, s);
        ++net->t;
        const float c1 = (float)(1.0 - std::pow((double)tp->beta1, (double)net->t));
        const float c2 = (float)(1.0 - std::pow((double)tp->beta2, (double)net->t));
        launch_mlp_reduce_adam(nblk, (int)net->P, net->partial.as<float>(), net->loss_partial.as<float>(), inv_n,
                               net->loss.as<float>() + step, net->params.as<float>(), net->m1.as<float>(),
                               net->m2.as<float>(), tp->lr, tp->beta1, tp->beta2, tp->eps, c1, c2, net->wb.p,
                               net->bb.as<float>(), s);
    }
    HIPCHK(ctx, hipGetLastError());
    if (int rc = check_flag(ctx, s, "sdm_mlp_train")) return rc;
    if (loss_curve)
        HIPCHK(ctx, hipMemcpy(loss_curve, net->loss.p, (size_t)tp->steps * sizeof(float), hipMemcpyDeviceToHost));
    return SDM_OK;
}

int sdm_mlp_infer(sdm_mlp *net, int64_t m, const float *tuples, const int32_t *panes, float *out, void *hip_stream)
{
    if (!net) return SDM_E_INVALID;
    sdm_context *ctx = net->ctx;
    if (int rc = mlp_check(net, m, tuples, panes)) return rc;
    if (m == 0) return SDM_OK;
    if (!out) return fail(ctx, SDM_E_INVALID, "null output");
    HIPCHK(ctx, hipSetDevice(ctx->device));
    hipStream_t s = (hipStream_t)hip_stream;
    HIPCHK(ctx, ctx->flag.ensure(sizeof(int)));
    launch_zero_i32(ctx->flag.as<int>(), 1, s);
    launch_mlp_pack(net->params.as<float>(), net->wb.p, net->bb.as<float>(), s);
    launch_mlp_infer((uint32_t)m, net->n_panes, tuples, panes, net->wb.p, net->bb.as<float>(),
                     net->params.as<float>() + mlp_net_params(), out, ctx->flag.as<int>(), ctx->num_cu, s);
    HIPCHK(ctx, hipGetLastError());
    return check_flag(ctx, s, "sdm_mlp_infer");
}

int sdm_mlp_error_table(sdm_mlp *net, int64_t m, const float *tuples, const int32_t *panes, const float *target,
                        const int32_t *dims, float *table, void *hip_stream)
{
    if (!net) return SDM_E_INVALID;
    sdm_context *ctx = net->ctx;
    if (int rc = mlp_check(net, m, tuples, panes)) return rc;
    if (!dims || !table || (m > 0 && !target)) return fail(ctx, SDM_E_INVALID, "null argument");
    for (int a = 0; a < 3; ++a)
        if (dims[a] < 1 || dims[a] > 1024) return fail(ctx, SDM_E_INVALID, "dims must be in [1, 1024]");
    if ((int64_t)net->n_panes * dims[0] * dims[1] * dims[2] > (1 << 24))
        return fail(ctx, SDM_E_INVALID, "error table too large");
    HIPCHK(ctx, hipSetDevice(ctx->device));
    hipStream_t s = (hipStream_t)hip_stream;
    HIPCHK(ctx, ctx->flag.ensure(sizeof(int)));
    HIPCHK(ctx, ctx->mc_acc.ensure(3 * (size_t)std::max<int64_t>(m, 1) * sizeof(float)));
    launch_zero_i32(ctx->flag.as<int>(), 1, s);
    float *y = ctx->mc_acc.as<float>();
    if (m > 0) {
        launch_mlp_pack(net->params.as<float>(), net->wb.p, net->bb.as<float>(), s);
        launch_mlp_infer((uint32_t)m, net->n_panes, tuples, panes, net->wb.p, net->bb.as<float>(),
                         net->params.as<float>() + mlp_net_params(), y, ctx->flag.as<int>(), ctx->num_cu, s);
    }
    const int d[3] = {dims[0], dims[1], dims[2]};
    launch_err_cells((uint32_t)m, tuples, panes, y, target, net->n_panes, d, table, ctx->flag.as<int>(), s);
    HIPCHK(ctx, hipGetLastError());
    return check_flag(ctx, s, "sdm_mlp_error_table");
}

int sdm_debug_mfma(sdm_context *ctx, const float *A32, const float *B32, float *C32, const float *A16,
                   const float *B16, float *C16, void *hip_stream)
{
    if (!ctx) return SDM_E_INVALID;
    if (!A32 || !B32 || !C32 || !A16 || !B16 || !C16) return fail(ctx, SDM_E_INVALID, "null array");
    HIPCHK(ctx, hipSetDevice(ctx->device));
    hipStream_t s = (hipStream_t)hip_stream;
    launch_mfma_probe(A32, B32, C32, A16, B16, C16, s);
    HIPCHK(ctx, hipGetLastError());
    HIPCHK(ctx, hipStreamSynchronize(s));
    return SDM_OK;
}

}  // extern "C"
