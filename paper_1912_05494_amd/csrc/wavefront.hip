// wavefront.hip -- kernels of the spectral wavefront path tracer (gfx950).
//
// A path carries one spectral band (a sub-domain of Sec. 4): all wavelengths
// of a (pixel, sample) draw the same random numbers, and thin-slab glass
// bends no wavelength differently, so they follow one ray until a glass
// vertex sends some wavelengths to reflection and others to transmission;
// then the path forks (wavelengths are still independent, so the image is
// the same as tracing each wavelength alone).  Per-wavelength path weights
// live in the path pool; queues hold pool slots.  One step of the loop of
// Sec. 3.1 is: closest hit -> shade (light sum of eq. (3) via a shadow
// record, reflect/refract, compaction) -> shadow rays.
#include <hip/hip_runtime.h>

#include <climits>

#include "sdm_dev.hpp"
#include "wavefront.hpp"

namespace sdm {

// ---------------------------------------------------------------------------
// Traversal
// ---------------------------------------------------------------------------
constexpr int kLdsNodes = 256;    // BVH prefix staged in LDS (16 KB)
constexpr int kBlock = 256;

struct Stack {
    int32_t *lds;       // [kLdsStack][kBlock]
    int32_t *glob;      // overflow, [(level - kLdsStack) * gstride + gtid]
    uint32_t gtid, gstride;
    int sp;
    __device__ __forceinline__ void push(int32_t v)
    {
        if (sp < kLdsStack) lds[sp * kBlock + threadIdx.x] = v;
        else glob[(size_t)(sp - kLdsStack) * gstride + gtid] = v;
        ++sp;
    }
    __device__ __forceinline__ int32_t pop()
    {
        --sp;
        return sp < kLdsStack ? lds[sp * kBlock + threadIdx.x]
                              : glob[(size_t)(sp - kLdsStack) * gstride + gtid];
    }
};

struct NodeView {
    float lo0[3], hi0[3], lo1[3], hi1[3];
    int32_t c0, c1, n0, n1;
};

__device__ __forceinline__ NodeView load_node(const float4 *lds_nodes, int n_lds, const BvhNode *nodes, int i)
{
    const float4 *p = (i < n_lds) ? lds_nodes + 4 * i : reinterpret_cast<const float4 *>(nodes) + 4 * (size_t)i;
    const float4 a = p[0], b = p[1], c = p[2], d = p[3];
    NodeView v;
    v.lo0[0] = a.x; v.lo0[1] = a.y; v.lo0[2] = a.z; v.hi0[0] = a.w;
    v.hi0[1] = b.x; v.hi0[2] = b.y; v.lo1[0] = b.z; v.lo1[1] = b.w;
    v.lo1[2] = c.x; v.hi1[0] = c.y; v.hi1[1] = c.z; v.hi1[2] = c.w;
    v.c0 = __float_as_int(d.x); v.c1 = __float_as_int(d.y);
    v.n0 = __float_as_int(d.z); v.n1 = __float_as_int(d.w);
    return v;
}

// Stage the BVH prefix of `sc` in LDS (whole block participates).
__device__ __forceinline__ int stage_nodes(float4 *lds_nodes, const SceneDev &sc)
{
    const int n = min(sc.n_nodes, kLdsNodes);
    const float4 *src = reinterpret_cast<const float4 *>(sc.nodes);
    for (int i = threadIdx.x; i < 4 * n; i += blockDim.x) lds_nodes[i] = src[i];
    __syncthreads();
    return n;
}

template <class R>
__device__ __forceinline__ R teps_of(const SceneDev &sc)
{
    return sizeof(R) == 4 ? R(sc.teps_f) : R(sc.teps_d);
}

// Closest hit.  Ties in t go to the smaller caller triangle index, so the
// result does not depend on the tree.  `skip` is a leaf-order index.
template <class R>
__device__ void closest_hit(const SceneDev &sc, const float4 *lds_nodes, int n_lds, Stack &st, V3<R> o,
                            V3<R> d, int32_t skip, R &tb, int32_t &trib, R &ub, R &vb, uint32_t &nodes,
                            uint32_t &tests)
{
    tb = R(INFINITY);
    trib = -1;
    ub = vb = R(0);
    if (sc.n_nodes == 0) return;
    int32_t orig_b = INT_MAX;
    const V3<R> inv = safe_inv(d);
    const R teps = teps_of<R>(sc);
    st.sp = 0;
    int cur = 0;
    auto leaf = [&](int first, int cnt) {
        tests += (uint32_t)cnt;
        for (int i = first; i < first + cnt; ++i) {
            if (i == skip) continue;
            const TriDev tr = sc.tris[i];
            R t, u, v;
            if (!tri_hit(o, d, from4<R>(tr.a), from4<R>(tr.b), from4<R>(tr.c), t, u, v)) continue;
            if (!(t > teps)) continue;
            const int32_t orig = __float_as_int(tr.a.w);
            if (t < tb || (t == tb && orig < orig_b)) {
                tb = t; trib = i; ub = u; vb = v; orig_b = orig;
            }
        }
    };
    for (;;) {
        const NodeView nv = load_node(lds_nodes, n_lds, sc.nodes, cur);
        ++nodes;
        R tn0, tn1;
        bool h0 = (nv.n0 > 0 || nv.c0 > 0) && box_hit(nv.lo0, nv.hi0, o, inv, teps, tb, tn0);
        bool h1 = (nv.n1 > 0 || nv.c1 > 0) && box_hit(nv.lo1, nv.hi1, o, inv, teps, tb, tn1);
        if (h0 && nv.n0 > 0) { leaf(nv.c0, nv.n0); h0 = false; }
        if (h1 && nv.n1 > 0) { leaf(nv.c1, nv.n1); h1 = false; }
        if (h0 && h1) {
            const bool first0 = tn0 <= tn1;
            st.push(first0 ? nv.c1 : nv.c0);
            cur = first0 ? nv.c0 : nv.c1;
        } else if (h0) {
            cur = nv.c0;
        } else if (h1) {
            cur = nv.c1;
        } else {
            if (st.sp == 0) break;
            cur = st.pop();
        }
    }
}

// Any-hit walk toward +infinity.  Returns true when an opaque triangle is
// crossed; calls on_glass(leaf_index, u, v) for every pane crossed.
template <class R, class F>
__device__ bool shadow_walk(const SceneDev &sc, const float4 *lds_nodes, int n_lds, Stack &st, V3<R> o,
                            V3<R> d, int32_t skip, F &&on_glass, uint32_t &nodes, uint32_t &tests)
{
    if (sc.n_nodes == 0) return false;
    const V3<R> inv = safe_inv(d);
    const R teps = teps_of<R>(sc);
    const R tinf = R(INFINITY);
    st.sp = 0;
    int cur = 0;
    for (;;) {
        const NodeView nv = load_node(lds_nodes, n_lds, sc.nodes, cur);
        ++nodes;
        R tn0, tn1;
        bool h0 = (nv.n0 > 0 || nv.c0 > 0) && box_hit(nv.lo0, nv.hi0, o, inv, teps, tinf, tn0);
        bool h1 = (nv.n1 > 0 || nv.c1 > 0) && box_hit(nv.lo1, nv.hi1, o, inv, teps, tinf, tn1);
#pragma unroll
        for (int w = 0; w < 2; ++w) {
            const int cnt = w ? nv.n1 : nv.n0;
            const bool hh = w ? h1 : h0;
            if (!(hh && cnt > 0)) continue;
            const int first = w ? nv.c1 : nv.c0;
            tests += (uint32_t)cnt;
            for (int i = first; i < first + cnt; ++i) {
                if (i == skip) continue;
                const TriDev tr = sc.tris[i];
                R t, u, v;
                if (!tri_hit(o, d, from4<R>(tr.a), from4<R>(tr.b), from4<R>(tr.c), t, u, v)) continue;
                if (!(t > teps)) continue;
                if (sc.mat_type[__float_as_int(tr.b.w)] == 0) return true;
                on_glass(i, u, v);
            }
            if (w) h1 = false; else h0 = false;
        }
        if (h0 && h1) {
            st.push(nv.c1);
            cur = nv.c0;
        } else if (h0) {
            cur = nv.c0;
        } else if (h1) {
            cur = nv.c1;
        } else {
            if (st.sp == 0) break;
            cur = st.pop();
        }
    }
    return false;
}

template <class R>
__device__ __forceinline__ V3<R> tri_normal(const TriDev &tr)
{
    const V3<R> p0 = from4<R>(tr.a), p1 = from4<R>(tr.b), p2 = from4<R>(tr.c);
    return normalize(cross(p1 - p0, p2 - p0));
}

template <class R>
__device__ __forceinline__ R pane_thickness(const SceneDev &sc, int leaf, R u, R v)
{
    if (!sc.has_vthick) return R(sc.mat_thick[__float_as_int(sc.tris[leaf].b.w)]);
    const float4 th = sc.thick[leaf];
    return (R(1) - u - v) * R(th.x) + u * R(th.y) + v * R(th.z);
}

__device__ __forceinline__ Stack make_stack(int32_t *lds_stack, int32_t *gstack)
{
    Stack st;
    st.lds = lds_stack;
    st.glob = gstack;
    st.gtid = blockIdx.x * blockDim.x + threadIdx.x;
    st.gstride = gridDim.x * blockDim.x;
    st.sp = 0;
    return st;
}

// ---------------------------------------------------------------------------
// Camera rays (Sec. 3.1: a ray from each pixel).  Image point ((i + u0) / W,
// (j + u1) / H), row j from the top; pinhole through the unit-distance image
// plane, or orthographic rays along the view axis.
// ---------------------------------------------------------------------------
template <class R>
__global__ void __launch_bounds__(kBlock) k_generate(const JobDev *jobs, const BandDev *bands,
                                                     const ItemDev *items, int32_t n_items, Work<R> w,
                                                     uint64_t r0, uint32_t n, int cur)
{
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        w.cnt->qcount[cur] = n;
        w.cnt->fork_next = w.primary_cap;
    }
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
        w.ox[i] = o.x; w.oy[i] = o.y; w.oz[i] = o.z;
        w.dx[i] = d.x; w.dy[i] = d.y; w.dz[i] = d.z;
        w.pix[i] = pixel;
        w.smp[i] = smp;
        w.aux[i] = pack_aux(0, it.band, bd.job);
        w.skip[i] = -1;
        for (int j = 0; j < bd.nb; ++j) w.beta[(size_t)j * w.cap + i] = R(1);
        w.q[cur][i] = i;
    }
}

// ---------------------------------------------------------------------------
// Closest-hit traversal of the current queue.
// ---------------------------------------------------------------------------
template <class R>
__global__ void __launch_bounds__(kBlock) k_trace(const JobDev *jobs, Work<R> w, int cur, int lds_job)
{
    __shared__ float4 s_nodes[4 * kLdsNodes];
    __shared__ int32_t s_stack[kLdsStack * kBlock];
    const uint32_t count = w.cnt->qcount[cur];
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        w.cnt->qcount[cur ^ 1] = 0;
        w.cnt->scount = 0;
        w.cnt->closest += count;
    }
    const int n_lds = lds_job >= 0 ? stage_nodes(s_nodes, jobs[lds_job].sc) : 0;
    Stack st = make_stack(s_stack, w.gstack);
    const uint32_t stride = gridDim.x * blockDim.x;
    uint32_t n_nodes = 0, n_tests = 0;
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < count; i += stride) {
        const uint32_t s = w.q[cur][i];
        const int job = (int)(w.aux[s] >> kAuxJobShift);
        const SceneDev &sc = jobs[job].sc;
        const V3<R> o = {w.ox[s], w.oy[s], w.oz[s]}, d = {w.dx[s], w.dy[s], w.dz[s]};
        R t, u, v;
        int32_t tri;
        closest_hit(sc, s_nodes, job == lds_job ? n_lds : 0, st, o, d, w.skip[s], t, tri, u, v, n_nodes, n_tests);
        w.ht[i] = t; w.htri[i] = tri; w.hu[i] = u; w.hv[i] = v;
    }
    if (n_nodes) {
        atomicAdd(&w.cnt->nodes[0], (unsigned long long)n_nodes);
        atomicAdd(&w.cnt->tris[0], (unsigned long long)n_tests);
    }
}

// ---------------------------------------------------------------------------
// Shade: misses add the sky, Lambert vertices emit a shadow record (eq. (3))
// and bounce, glass vertices reflect or pass per wavelength; survivors are
// compacted into the next queue.
// ---------------------------------------------------------------------------
template <class R>
__global__ void __launch_bounds__(kBlock) k_shade(const JobDev *jobs, const BandDev *bands, Work<R> w, int cur)
{
    const uint32_t count = w.cnt->qcount[cur];
    const uint32_t *qin = w.q[cur];
    uint32_t *qout = w.q[cur ^ 1];
    const size_t cap = w.cap;
    const uint32_t lane = lane_id();
    const uint32_t wave = (blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const uint32_t nwaves = (gridDim.x * blockDim.x) >> 6;
    const R inv_pi = R(0.31830988618379067);
    for (uint32_t base = wave * 64; base < count; base += nwaves * 64) {
        const uint32_t i = base + lane;
        const bool active = i < count;
        uint32_t s = 0, aux = 0, pix = 0;
        int32_t tri = -1;
        int kind = -1;            // 0 miss, 1 lambert, 2 glass
        bool last = true, want_shadow = false;
        V3<R> x = {R(0), R(0), R(0)}, dnew = x, drefl = x, ns = x;
        R cs = R(0), cos_i = R(0), thick = R(0), u0 = R(0);
        int mat = 0, job = 0, band = 0, depth = 0;
        const JobDev *jb = nullptr;
        BandDev bd = {0, 0, 0, 0};
        if (active) {
            s = qin[i];
            aux = w.aux[s];
            pix = w.pix[s];
            depth = (int)(aux & 0xffu);
            band = (int)((aux >> kAuxBandShift) & ((1u << kAuxBandBits) - 1u));
            job = (int)(aux >> kAuxJobShift);
            jb = &jobs[job];
            bd = bands[band];
            tri = w.htri[i];
            last = depth >= jb->max_depth - 1;
            if (tri < 0) {
                kind = 0;
            } else {
                const V3<R> o = {w.ox[s], w.oy[s], w.oz[s]}, d = {w.dx[s], w.dy[s], w.dz[s]};
                const R t = w.ht[i];
                x = o + t * d;
                const TriDev tr = jb->sc.tris[tri];
                mat = __float_as_int(tr.b.w);
                const V3<R> ng = tri_normal<R>(tr);
                const uint4 rr = vertex_draws(jb->seed, jb->job_word, pix, w.smp[s], depth, 0);
                u0 = u01<R>(rr.x);
                if (jb->sc.mat_type[mat] == 0) {
                    kind = 1;
                    ns = dot(ng, d) > R(0) ? R(-1) * ng : ng;
                    const V3<R> sun = {R(jb->sc.sun[0]), R(jb->sc.sun[1]), R(jb->sc.sun[2])};
                    cs = dot(ns, sun);
                    want_shadow = cs > R(0);
                    if (!last) dnew = cosine_dir(ns, u01<R>(rr.y), u01<R>(rr.z));
                } else {
                    kind = 2;
                    cos_i = fabs(dot(d, ng));
                    thick = pane_thickness<R>(jb->sc, tri, w.hu[i], w.hv[i]);
                    dnew = d;
                    drefl = d - (R(2) * dot(d, ng)) * ng;
                }
            }
        }
        // shadow records (one atomic per wave)
        const uint32_t sslot = wave_reserve(want_shadow, &w.cnt->scount);
        bool keep = false, fork = false;
        uint32_t m0 = 0, m1 = 0, m2 = 0, m3 = 0;   // reflected-wavelength mask
        if (active) {
            const int nl = jb->nl;
            const R *E = (const R *)jb->E;
            const R thr = R(jb->beta_thr);
            if (kind == 0) {
                const R *Ls = (const R *)jb->Lsky;
                double *acc = w.acc + jb->acc_off + (size_t)pix * nl + bd.l0;
                for (int j = 0; j < bd.nb; ++j) {
                    const R b = w.beta[(size_t)j * cap + s];
                    if (b != R(0)) unsafeAtomicAdd(acc + j, (double)(b * Ls[bd.l0 + j]));
                }
            } else if (kind == 1) {
                const R *rho = (const R *)jb->rho + (size_t)mat * nl + bd.l0;
                bool any = false;
                if (want_shadow) {
                    w.sx[sslot] = x.x; w.sy[sslot] = x.y; w.sz[sslot] = x.z;
                    w.sskip[sslot] = tri;
                    w.spix[sslot] = pix;
                    w.saux[sslot] = aux;
                }
                for (int j = 0; j < bd.nb; ++j) {
                    const R b = w.beta[(size_t)j * cap + s];
                    const R rj = rho[j];
                    if (want_shadow) w.contrib[(size_t)j * cap + sslot] = b * rj * inv_pi * E[bd.l0 + j] * cs;
                    if (!last) {
                        R bn = b * rj;
                        if (bn < thr) bn = R(0);
                        w.beta[(size_t)j * cap + s] = bn;
                        any |= bn != R(0);
                    }
                }
                keep = !last && any;
            } else if (kind == 2 && !last) {
                const R *nn = (const R *)jb->n + (size_t)mat * nl + bd.l0;
                const R *kk = (const R *)jb->k + (size_t)mat * nl + bd.l0;
                const R *tt = (const R *)jb->tint + (size_t)mat * nl + bd.l0;
                const R *lam = (const R *)jb->lam + bd.l0;
                bool anyR = false, anyT = false;
                for (int j = 0; j < bd.nb; ++j) {
                    const R b = w.beta[(size_t)j * cap + s];
                    R Rr = R(0), Tt = R(0), bn = R(0);
                    bool refl = false;
                    if (b != R(0)) {
                        slab_RT<R>(cos_i, lam[j], thick, nn[j], kk[j], tt[j], Rr, Tt);
                        const R rt = Rr + Tt;
                        refl = rt > R(0) && u0 < Rr / rt;
                        bn = b * rt;
                        if (bn < thr) bn = R(0);
                    }
                    w.beta[(size_t)j * cap + s] = bn;
                    if (bn != R(0)) {
                        if (refl) {
                            anyR = true;
                            const uint32_t bit = 1u << (j & 31);
                            if (j < 32) m0 |= bit; else if (j < 64) m1 |= bit; else if (j < 96) m2 |= bit; else m3 |= bit;
                        } else {
                            anyT = true;
                        }
                    }
                }
                keep = anyR || anyT;
                fork = anyR && anyT;
                if (anyR && !anyT) dnew = drefl;   // whole band reflects: no fork
            }
        }
        // fork slots in the pool
        uint32_t fslot = wave_reserve(fork, &w.cnt->fork_next);
        {
            const uint64_t mfk = __ballot(fork);
            if (mfk && (int)lane == __ffsll((unsigned long long)mfk) - 1)
                atomicAdd(&w.cnt->forks, (unsigned long long)__popcll(mfk));
        }
        if (fork && fslot >= w.cap) {
            w.cnt->overflow = 1;
            fork = false;
        }
        if (active && fork) {
            for (int j = 0; j < bd.nb; ++j) {
                const uint32_t word = j < 32 ? m0 : j < 64 ? m1 : j < 96 ? m2 : m3;
                const R b = w.beta[(size_t)j * cap + s];
                const bool refl = (word >> (j & 31)) & 1u;
                w.beta[(size_t)j * cap + fslot] = refl ? b : R(0);
                if (refl) w.beta[(size_t)j * cap + s] = R(0);
            }
            w.ox[fslot] = x.x; w.oy[fslot] = x.y; w.oz[fslot] = x.z;
            w.dx[fslot] = drefl.x; w.dy[fslot] = drefl.y; w.dz[fslot] = drefl.z;
            w.pix[fslot] = pix;
            w.smp[fslot] = w.smp[s];
            w.aux[fslot] = aux + 1u;
            w.skip[fslot] = tri;
        }
        if (active && keep) {
            w.ox[s] = x.x; w.oy[s] = x.y; w.oz[s] = x.z;
            w.dx[s] = dnew.x; w.dy[s] = dnew.y; w.dz[s] = dnew.z;
            w.aux[s] = aux + 1u;
            w.skip[s] = tri;
        }
        // compaction of survivors and forks into the next queue
        const uint64_t mk = __ballot(keep), mf = __ballot(fork);
        const uint32_t nk = (uint32_t)__popcll(mk), nf = (uint32_t)__popcll(mf);
        const uint64_t lt = (1ull << lane) - 1ull;
        uint32_t qbase = 0;
        if (nk + nf) {
            const int leader = __ffsll((unsigned long long)(mk | mf)) - 1;
            if ((int)lane == leader) qbase = atomicAdd(&w.cnt->qcount[cur ^ 1], nk + nf);
            qbase = __shfl(qbase, leader);
        }
        if (keep) qout[qbase + (uint32_t)__popcll(mk & lt)] = s;
        if (fork) qout[qbase + nk + (uint32_t)__popcll(mf & lt)] = fslot;
    }
}

// ---------------------------------------------------------------------------
// Shadow rays toward the sun: an opaque hit ends the record; every pane
// crossed multiplies in its slab transmittance at the sun angle.  The
// product is accumulated in FP64.
// ---------------------------------------------------------------------------
template <class R>
__global__ void __launch_bounds__(kBlock) k_shadow(const JobDev *jobs, const BandDev *bands, Work<R> w, int lds_job)
{
    __shared__ float4 s_nodes[4 * kLdsNodes];
    __shared__ int32_t s_stack[kLdsStack * kBlock];
    const uint32_t count = w.cnt->scount;
    if (blockIdx.x == 0 && threadIdx.x == 0) w.cnt->shadow += count;
    const int n_lds = lds_job >= 0 ? stage_nodes(s_nodes, jobs[lds_job].sc) : 0;
    Stack st = make_stack(s_stack, w.gstack);
    const size_t cap = w.cap;
    const uint32_t stride = gridDim.x * blockDim.x;
    constexpr int G = 4;
    uint32_t n_nodes = 0, n_tests = 0;
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < count; i += stride) {
        const uint32_t aux = w.saux[i];
        const int job = (int)(aux >> kAuxJobShift);
        const int band = (int)((aux >> kAuxBandShift) & ((1u << kAuxBandBits) - 1u));
        const JobDev &jb = jobs[job];
        const BandDev bd = bands[band];
        const int nl = jb.nl;
        const R *nn_t = (const R *)jb.n, *kk_t = (const R *)jb.k, *tt_t = (const R *)jb.tint;
        const R *lam = (const R *)jb.lam + bd.l0;
        const V3<R> o = {w.sx[i], w.sy[i], w.sz[i]};
        const V3<R> sun = {R(jb.sc.sun[0]), R(jb.sc.sun[1]), R(jb.sc.sun[2])};
        // panes crossed, kept in registers; folded into contrib when full
        R gc[G], gd[G];
        int gm[G];
        int ng = 0;
        auto fold = [&]() {
            for (int j = 0; j < bd.nb; ++j) {
                R T = w.contrib[(size_t)j * cap + i];
                for (int g = 0; g < ng; ++g) {
                    R Rr, Tt;
                    const size_t mo = (size_t)gm[g] * nl + bd.l0 + j;
                    slab_RT<R>(gc[g], lam[j], gd[g], nn_t[mo], kk_t[mo], tt_t[mo], Rr, Tt);
                    T *= Tt;
                }
                w.contrib[(size_t)j * cap + i] = T;
            }
            ng = 0;
        };
        const bool occluded = shadow_walk<R>(jb.sc, s_nodes, job == lds_job ? n_lds : 0, st, o, sun, w.sskip[i],
                                             [&](int leaf, R u, R v) {
                                                 const TriDev tr = jb.sc.tris[leaf];
                                                 if (ng == G) fold();
                                                 gc[ng] = fabs(dot(sun, tri_normal<R>(tr)));
                                                 gd[ng] = pane_thickness<R>(jb.sc, leaf, u, v);
                                                 gm[ng] = __float_as_int(tr.b.w);
                                                 ++ng;
                                             }, n_nodes, n_tests);
        if (occluded) continue;
        double *acc = w.acc + jb.acc_off + (size_t)w.spix[i] * nl + bd.l0;
        for (int j = 0; j < bd.nb; ++j) {
            R T = w.contrib[(size_t)j * cap + i];
            for (int g = 0; g < ng; ++g) {
                R Rr, Tt;
                const size_t mo = (size_t)gm[g] * nl + bd.l0 + j;
                slab_RT<R>(gc[g], lam[j], gd[g], nn_t[mo], kk_t[mo], tt_t[mo], Rr, Tt);
                T *= Tt;
            }
            if (T != R(0)) unsafeAtomicAdd(acc + j, (double)T);
        }
    }
    if (n_nodes) {
        atomicAdd(&w.cnt->nodes[1], (unsigned long long)n_nodes);
        atomicAdd(&w.cnt->tris[1], (unsigned long long)n_tests);
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
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < npix; p += stride) {
        double X = 0.0, Y = 0.0, Z = 0.0;
        const double *a = acc + p * nl;
        for (int l = 0; l < nl; ++l) {
            const double v = a[l] / spp;
            if (spec) spec[p * nl + l] = (float)v;
            const double wv = wts[l] * v;
            X += wv * cmf[3 * l];
            Y += wv * cmf[3 * l + 1];
            Z += wv * cmf[3 * l + 2];
        }
        if (xyz) {
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

__global__ void k_zero_counters(Counters *c)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        c->qcount[0] = c->qcount[1] = 0;
        c->scount = 0;
        c->fork_next = 0;
        c->overflow = 0;
        c->closest = c->shadow = c->forks = 0;
        c->nodes[0] = c->nodes[1] = c->tris[0] = c->tris[1] = 0;
    }
}

// Linear interpolation of a table (tab_x[n_tab], tab_y[n_tab]) at xs[nl],
// held constant beyond the ends; rows of `rows` tables.
template <class R>
__global__ void k_resample(const float *tab_x, int n_tab, const float *tab_y, int rows, const float *xs,
                           int nl, R *out)
{
    const int total = rows * nl;
    for (int id = blockIdx.x * blockDim.x + threadIdx.x; id < total; id += gridDim.x * blockDim.x) {
        const int r = id / nl, l = id % nl;
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

__global__ void __launch_bounds__(kBlock) k_debug_intersect(SceneDev sc, int64_t m, const float *o, const float *d,
                                                            const int32_t *skip, const int32_t *orig_to_leaf,
                                                            float *t, int32_t *tri, float *uv,
                                                            int32_t *gstack)
{
    __shared__ float4 s_nodes[4 * kLdsNodes];
    __shared__ int32_t s_stack[kLdsStack * kBlock];
    const int n_lds = stage_nodes(s_nodes, sc);
    Stack st = make_stack(s_stack, gstack);
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < m; i += stride) {
        const V3<float> oo = {o[3 * i], o[3 * i + 1], o[3 * i + 2]}, dd = {d[3 * i], d[3 * i + 1], d[3 * i + 2]};
        const int32_t sk = (skip && skip[i] >= 0 && skip[i] < sc.nt) ? orig_to_leaf[skip[i]] : -1;
        float tt, u, v;
        int32_t leaf;
        uint32_t nn = 0, nt = 0;
        closest_hit<float>(sc, s_nodes, n_lds, st, oo, dd, sk, tt, leaf, u, v, nn, nt);
        t[i] = tt;
        tri[i] = leaf >= 0 ? __float_as_int(sc.tris[leaf].a.w) : -1;
        uv[2 * i] = u;
        uv[2 * i + 1] = v;
    }
}

__global__ void __launch_bounds__(kBlock) k_debug_shadow(SceneDev sc, int64_t m, const float *o, const int32_t *skip,
                                                         const int32_t *orig_to_leaf, float lambda_nm,
                                                         const float *n_at, const float *k_at, const float *t_at,
                                                         float *T, int32_t *gstack)
{
    __shared__ float4 s_nodes[4 * kLdsNodes];
    __shared__ int32_t s_stack[kLdsStack * kBlock];
    const int n_lds = stage_nodes(s_nodes, sc);
    Stack st = make_stack(s_stack, gstack);
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    const V3<float> sun = {sc.sun[0], sc.sun[1], sc.sun[2]};
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < m; i += stride) {
        const V3<float> oo = {o[3 * i], o[3 * i + 1], o[3 * i + 2]};
        const int32_t sk = (skip && skip[i] >= 0 && skip[i] < sc.nt) ? orig_to_leaf[skip[i]] : -1;
        float prod = 1.0f;
        uint32_t nn = 0, nt = 0;
        const bool occ = shadow_walk<float>(sc, s_nodes, n_lds, st, oo, sun, sk, [&](int leaf, float u, float v) {
            const TriDev tr = sc.tris[leaf];
            const int mt = __float_as_int(tr.b.w);
            float Rr, Tt;
            slab_RT<float>(fabsf(dot(sun, tri_normal<float>(tr))), lambda_nm, pane_thickness<float>(sc, leaf, u, v),
                           n_at[mt], k_at[mt], t_at[mt], Rr, Tt);
            prod *= Tt;
        }, nn, nt);
        T[i] = occ ? 0.0f : prod;
    }
}

// ---------------------------------------------------------------------------
// Host launchers
// ---------------------------------------------------------------------------
template <class R>
void launch_generate(const JobDev *jobs, const BandDev *bands, const ItemDev *items, int n_items, const Work<R> &w,
                     uint64_t r0, uint32_t n, int cur, int grid, hipStream_t s)
{
    hipLaunchKernelGGL(k_generate<R>, dim3(grid), dim3(kBlock), 0, s, jobs, bands, items, n_items, w, r0, n, cur);
}
template <class R>
void launch_trace(const JobDev *jobs, const Work<R> &w, int cur, int lds_job, int grid, hipStream_t s)
{
    hipLaunchKernelGGL(k_trace<R>, dim3(grid), dim3(kBlock), 0, s, jobs, w, cur, lds_job);
}
template <class R>
void launch_shade(const JobDev *jobs, const BandDev *bands, const Work<R> &w, int cur, int grid, hipStream_t s)
{
    hipLaunchKernelGGL(k_shade<R>, dim3(grid), dim3(kBlock), 0, s, jobs, bands, w, cur);
}
template <class R>
void launch_shadow(const JobDev *jobs, const BandDev *bands, const Work<R> &w, int lds_job, int grid, hipStream_t s)
{
    hipLaunchKernelGGL(k_shadow<R>, dim3(grid), dim3(kBlock), 0, s, jobs, bands, w, lds_job);
}
template <class R>
void launch_resample(const float *tab_x, int n_tab, const float *tab_y, int rows, const float *xs, int nl, R *out,
                     hipStream_t s)
{
    const int total = rows * nl;
    const int grid = std::max(1, std::min(1024, (total + kBlock - 1) / kBlock));
    hipLaunchKernelGGL(k_resample<R>, dim3(grid), dim3(kBlock), 0, s, tab_x, n_tab, tab_y, rows, xs, nl, out);
}

void launch_finalize(const double *acc, int64_t npix, int nl, int spp, const double *wts, const double *cmf,
                     float *spec, double *xyz, hipStream_t s)
{
    const int grid = (int)std::max<int64_t>(1, std::min<int64_t>(8192, (npix + kBlock - 1) / kBlock));
    hipLaunchKernelGGL(k_finalize, dim3(grid), dim3(kBlock), 0, s, acc, npix, nl, spp, wts, cmf, spec, xyz);
}
void launch_zero_f64(double *a, int64_t n, hipStream_t s)
{
    const int grid = (int)std::max<int64_t>(1, std::min<int64_t>(16384, (n + kBlock - 1) / kBlock));
    hipLaunchKernelGGL(k_zero_f64, dim3(grid), dim3(kBlock), 0, s, a, n);
}
void launch_zero_counters(Counters *c, hipStream_t s)
{
    hipLaunchKernelGGL(k_zero_counters, dim3(1), dim3(64), 0, s, c);
}
void launch_slab_eval(int64_t m, const float *c, const float *lam, const float *d, const float *n, const float *k,
                      const float *tint, float *R, float *T, hipStream_t s)
{
    const int grid = (int)std::max<int64_t>(1, std::min<int64_t>(8192, (m + kBlock - 1) / kBlock));
    hipLaunchKernelGGL(k_slab_eval, dim3(grid), dim3(kBlock), 0, s, m, c, lam, d, n, k, tint, R, T);
}
void launch_debug_intersect(const SceneDev &sc, int64_t m, const float *o, const float *d, const int32_t *skip,
                            const int32_t *orig_to_leaf, float *t, int32_t *tri, float *uv, int32_t *gstack,
                            int grid, hipStream_t s)
{
    hipLaunchKernelGGL(k_debug_intersect, dim3(grid), dim3(kBlock), 0, s, sc, m, o, d, skip, orig_to_leaf, t, tri,
                       uv, gstack);
}
void launch_debug_shadow(const SceneDev &sc, int64_t m, const float *o, const int32_t *skip,
                         const int32_t *orig_to_leaf, float lambda_nm, const float *n_at, const float *k_at,
                         const float *t_at, float *T, int32_t *gstack, int grid, hipStream_t s)
{
    hipLaunchKernelGGL(k_debug_shadow, dim3(grid), dim3(kBlock), 0, s, sc, m, o, skip, orig_to_leaf, lambda_nm, n_at,
                       k_at, t_at, T, gstack);
}

int block_size() { return kBlock; }

template <class R>
int occupancy_trace()
{
    int b = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&b, k_trace<R>, kBlock, 0) != hipSuccess) return 1;
    return std::max(1, b);
}
template <class R>
int occupancy_shade()
{
    int b = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&b, k_shade<R>, kBlock, 0) != hipSuccess) return 1;
    return std::max(1, b);
}

#define SDM_INSTANTIATE(R)                                                                                        \
    template void launch_generate<R>(const JobDev *, const BandDev *, const ItemDev *, int, const Work<R> &,      \
                                     uint64_t, uint32_t, int, int, hipStream_t);                                  \
    template void launch_trace<R>(const JobDev *, const Work<R> &, int, int, int, hipStream_t);                   \
    template void launch_shade<R>(const JobDev *, const BandDev *, const Work<R> &, int, int, hipStream_t);       \
    template void launch_shadow<R>(const JobDev *, const BandDev *, const Work<R> &, int, int, hipStream_t);      \
    template void launch_resample<R>(const float *, int, const float *, int, const float *, int, R *,             \
                                     hipStream_t);                                                                \
    template int occupancy_trace<R>();                                                                            \
    template int occupancy_shade<R>();

SDM_INSTANTIATE(float)
SDM_INSTANTIATE(double)

}  // namespace sdm
