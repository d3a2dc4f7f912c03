// surrogate.hip -- tables of the bubbly-glass slab by Monte Carlo and the
// BF16-MFMA surrogate network (gfx950).
//
// Slab walk: see bubbly_dev.hpp (entry interface with n + ik of eq. (1),
// walk inside at the pane's real index, Beer-Lambert over the glass length,
// Poisson air bubbles with exact sphere optics for the direction).
//
// Network: 12 -> 64 -> 64 -> 64 -> 3, ReLU, heads R, T = softmax over
// (o0, o1, 0), w = softplus(o2); loss = mean squared error over (R, T, w).
// Operands BF16, accumulation FP32, master weights FP32 (Adam).
#include <hip/hip_runtime.h>

#include <mutex>

#include "bubbly_dev.hpp"
#include "mlp_dev.hpp"
#include "surrogate.hpp"

namespace sdm {

__global__ void k_mfma_probe(const float *A32, const float *B32, float *C32, const float *A16, const float *B16,
                             float *C16)
{
    const int l = threadIdx.x, g = l / 16, c = l % 16;
    bf16x8 a, b;
    for (int j = 0; j < 8; ++j) {
        a[j] = (__bf16)A32[c * 32 + 8 * g + j];
        b[j] = (__bf16)B32[(8 * g + j) * 16 + c];
    }
    f32x4 d = {0, 0, 0, 0};
    d = mfma32(a, b, d);
    for (int r = 0; r < 4; ++r) C32[(4 * g + r) * 16 + c] = d[r];
    s16x4 a2, b2;
    for (int j = 0; j < 4; ++j) {
        a2[j] = bits((__bf16)A16[c * 16 + 4 * g + j]);
        b2[j] = bits((__bf16)B16[(4 * g + j) * 16 + c]);
    }
    f32x4 d2 = {0, 0, 0, 0};
    d2 = mfma16(a2, b2, d2);
    for (int r = 0; r < 4; ++r) C16[(4 * g + r) * 16 + c] = d2[r];
}

// ---------------------------------------------------------------------------
// Bubbly slab Monte Carlo
// ---------------------------------------------------------------------------
struct McOut {
    double R, T, A, dev2;
};

// One photon of a table tuple: entry interface with the complex index at
// lambda (eq. (1)) and the label s/p, then the walk inside.
template <class R>
__device__ McOut mc_photon(R cos_i, R lam, R d, R sigma, R n, R k, R tint, R n_ref, uint64_t seed, uint32_t tuple,
                           uint32_t ph)
{
    McOut o = {0, 0, 0, 0};
    const WalkStream ws = {seed, tuple, ph, 0, 0, false};
    R u[4];
    walk_draw<R>(ws, 0, 0, u);
    const int pol = u[1] < R(0.5) ? 0 : 1;
    R Rs, Rp;
    fresnel_sp<R>(cos_i, n, k, Rs, Rp);
    if (u[0] < (pol == 0 ? Rs : Rp)) {
        o.R = 1.0;
        return o;
    }
    const WalkOut<R> w = bubbly_walk<R>(ws, cos_i, d, sigma, n_ref, pol);
    if (w.kind == 0) {
        o.A = 1.0;
        return o;
    }
    const R alpha = R(12.566370614359172) * k / (lam * R(1e-6)) + tint;
    const R wt = exp(-alpha * w.L);
    if (w.kind == 2) {
        o.T = (double)wt;
        const R sin_i = sqrt(fmax(R(1) - cos_i * cos_i, R(0)));
        const R c = fmin(fmax(w.a.x * sin_i + w.a.z * cos_i, R(-1)), R(1));
        const R dev = acos(c);
        o.dev2 = (double)(wt * dev * dev);
    } else {
        o.R = (double)wt;
    }
    o.A = 1.0 - (double)wt;
    return o;
}

// One walk per (tuple, photon); FP64 sums per tuple in acc[tuple][4] =
// (R, T, A, T-weighted squared deviation).  Waves take 64 consecutive
// (tuple, photon) pairs; runs of one tuple are summed in the wave first.
template <class R>
__global__ void __launch_bounds__(256) k_slab_mc(uint32_t m, uint32_t nph, const float *cos_i, const float *lam,
                                                 const float *d, const float *rho, const float *n, const float *k,
                                                 const float *tint, const float *n_ref, double r2_mm, uint64_t seed,
                                                 uint32_t tuple0, double *acc)
{
    const uint64_t total = (uint64_t)m * nph;
    const uint32_t lane = lane_id();
    const uint64_t wave = (blockIdx.x * (uint64_t)blockDim.x + threadIdx.x) >> 6;
    const uint64_t nw = ((uint64_t)gridDim.x * blockDim.x) >> 6;
    for (uint64_t base = wave * 64; base < total; base += nw * 64) {
        const uint64_t i = base + lane;
        uint32_t t = 0xffffffffu;
        McOut o = {0, 0, 0, 0};
        if (i < total) {
            t = (uint32_t)(i / nph);
            const uint32_t ph = (uint32_t)(i % nph);
            const R sigma = R((double)rho[t] * 3.14159265358979323846 * r2_mm);   // rho pi <r^2>
            o = mc_photon<R>(R(cos_i[t]), R(lam[t]), R(d[t]), sigma, R(n[t]), R(k[t]), tint ? R(tint[t]) : R(0),
                             n_ref ? R(n_ref[t]) : R(n[t]), seed, tuple0 + t, ph);
        }
        // runs of lanes of the same tuple: segmented sums, one atomic per run
        const uint32_t prev = __shfl_up(t, 1);
        uint32_t start = (lane == 0 || prev != t) ? lane : 0u;
        for (int off = 1; off < 64; off <<= 1) {
            const uint32_t s = __shfl_up(start, off);
            if ((int)lane >= off) start = max(start, s);
        }
        double v[4] = {o.R, o.T, o.A, o.dev2};
        for (int off = 1; off < 64; off <<= 1) {
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const double x = __shfl_up(v[q], off);
                if (lane >= start + (uint32_t)off) v[q] += x;
            }
        }
        const uint32_t next = __shfl_down(t, 1);
        if ((lane == 63 || next != t) && t != 0xffffffffu)
            for (int q = 0; q < 4; ++q) unsafeAtomicAdd(acc + 4 * (size_t)t + q, v[q]);
    }
}

__global__ void k_slab_mc_out(uint32_t m, uint32_t nph, const double *acc, float *R, float *T, float *A, float *W)
{
    for (uint32_t t = blockIdx.x * blockDim.x + threadIdx.x; t < m; t += gridDim.x * blockDim.x) {
        const double *a = acc + 4 * (size_t)t;
        R[t] = (float)(a[0] / nph);
        T[t] = (float)(a[1] / nph);
        if (A) A[t] = (float)(a[2] / nph);
        W[t] = a[1] > 0.0 ? (float)(sqrt(a[3] / a[1]) * 0.7071067811865476) : 0.0f;
    }
}

__global__ void k_zero_f64s(double *a, size_t n)
{
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) a[i] = 0.0;
}

// dW[out][in] += sum_s dZ[s][out] H[s][in] over the 16 samples (k = 16),
// for out tiles [0, nto) and in tiles [0, nti); atomically into LDS.
__device__ __forceinline__ void accum_dw(const __bf16 *dZ, int ldz, int nto, const __bf16 *H, int ldh, int nti,
                                         float *gW, int ldg, int out_max, int in_max)
{
    const int l = lane_id(), g = l / 16, c = l % 16;
    for (int to = 0; to < nto; ++to) {
        s16x4 a;
        for (int j = 0; j < 4; ++j) a[j] = bits(dZ[(4 * g + j) * ldz + 16 * to + c]);
        for (int ti = 0; ti < nti; ++ti) {
            s16x4 bv;
            for (int j = 0; j < 4; ++j) bv[j] = bits(H[(4 * g + j) * ldh + 16 * ti + c]);
            f32x4 acc = {0, 0, 0, 0};
            acc = mfma16(a, bv, acc);
            for (int r = 0; r < 4; ++r) {
                const int o = 16 * to + 4 * g + r, i = 16 * ti + c;
                if (o < out_max && i < in_max) atomicAdd(gW + o * ldg + i, acc[r]);
            }
        }
    }
}

// dH[16][nti*16] = dZ[16][K] W[K][nti*16] with K = 16 * kq (W row-major
// [K][ldw]); then ReLU mask from Hm (> 0) into Zout (BF16); bias sums into gb.
__device__ __forceinline__ void back_dense(const __bf16 *dZ, int ldz, int kq, const __bf16 *W, int ldw, int nti,
                                           const __bf16 *Hm, int ldm, __bf16 *Zout, int ldo, float *gb, float *dx_out)
{
    const int l = lane_id(), g = l / 16, c = l % 16;
    for (int ti = 0; ti < nti; ++ti) {
        f32x4 acc = {0, 0, 0, 0};
        for (int kk = 0; kk < kq; ++kk) {
            s16x4 a, bv;
            for (int j = 0; j < 4; ++j) {
                a[j] = bits(dZ[c * ldz + 16 * kk + 4 * g + j]);
                bv[j] = bits(W[(16 * kk + 4 * g + j) * ldw + 16 * ti + c]);
            }
            acc = mfma16(a, bv, acc);
        }
        float colsum = 0.0f;
        for (int r = 0; r < 4; ++r) {
            const int s = 4 * g + r, i = 16 * ti + c;
            if (dx_out) {
                dx_out[s * 16 + c] = acc[r];
                continue;
            }
            const float z = (float)Hm[s * ldm + i] > 0.0f ? acc[r] : 0.0f;
            Zout[s * ldo + i] = (__bf16)z;
            colsum += z;
        }
        if (gb) atomicAdd(gb + 16 * ti + c, colsum);
    }
}

// Gradient of the mean loss over a batch of m samples (inv_n = 1 / m).  Each
// wave takes 16-sample tiles through the forward and backward passes; weight,
// bias and embedding gradients are summed per block in LDS (ds_add) and
// written as one row of P = 9347 + 8 n_panes values per block.
__global__ void __launch_bounds__(256) k_mlp_grad(uint32_t m, int n_panes, const float *tup, const int32_t *pane,
                                                  const float *target, const __bf16 *wb, const float *bb,
                                                  const float *E, float inv_n, float *partial, float *loss_partial,
                                                  int *bad)
{
    __shared__ NetLds net;
    __shared__ WaveBuf wbuf[4];
    __shared__ float gacc[kNetParams + 8 * kMaxPanes];
    __shared__ float lsum[4];
    const int P = kNetParams + 8 * n_panes;
    for (int i = threadIdx.x; i < P; i += blockDim.x) gacc[i] = 0.0f;
    load_net(net, wb, bb);
    WaveBuf &w = wbuf[threadIdx.x >> 6];
    const int l = lane_id();
    float my_loss = 0.0f;
    const uint32_t ntile = (m + 15) / 16;
    const uint32_t wave = (blockIdx.x * blockDim.x + threadIdx.x) >> 6, nw = (gridDim.x * blockDim.x) >> 6;
    for (uint32_t tile = wave; tile < ntile; tile += nw) {
        const uint32_t s0 = tile * 16;
        int my_pane = -1;   // -1: padding or an invalid pane index (reported in *bad)
        if (l < 16) {
            const uint32_t s = s0 + l;
            if (s < m) {
                my_pane = pane[s];
                if ((unsigned)my_pane >= (unsigned)n_panes) {
                    atomicOr(bad, 1);
                    my_pane = -1;
                }
            }
            if (my_pane >= 0) features(tup[4 * s], tup[4 * s + 1], tup[4 * s + 2], tup[4 * s + 3], E + 8 * my_pane,
                                       w.X0 + l * 32);
            else for (int e = 0; e < 32; ++e) w.X0[l * 32 + e] = (__bf16)0.0f;
        }
        wave_sync();
        forward_tile(net, w);
        // heads, loss and d loss / d o; padded samples get a zero gradient
        if (l < 16) {
            const uint32_t s = s0 + l;
            float go0 = 0, go1 = 0, go2 = 0;
            if (my_pane >= 0) {
                const float o0 = w.O[l * 16], o1 = w.O[l * 16 + 1], o2 = w.O[l * 16 + 2];
                float R, T, wl;
                heads(o0, o1, o2, R, T, wl);
                const float e0 = R - target[3 * s], e1 = T - target[3 * s + 1], e2 = wl - target[3 * s + 2];
                my_loss += e0 * e0 + e1 * e1 + e2 * e2;
                const float gR = 2.0f * e0 * inv_n, gT = 2.0f * e1 * inv_n, gw = 2.0f * e2 * inv_n;
                go0 = gR * R * (1.0f - R) - gT * T * R;
                go1 = -gR * R * T + gT * T * (1.0f - T);
                go2 = gw / (1.0f + expf(-o2));
                atomicAdd(gacc + kOffB4, go0);
                atomicAdd(gacc + kOffB4 + 1, go1);
                atomicAdd(gacc + kOffB4 + 2, go2);
            }
            for (int q = 0; q < 16; ++q) w.dO[l * 16 + q] = (__bf16)(q == 0 ? go0 : q == 1 ? go1 : q == 2 ? go2 : 0.0f);
        }
        wave_sync();
        // output layer: dW4 (3 x 64) and dZ3 = (dO W4) masked by H3
        accum_dw(w.dO, 16, 1, w.H3, 64, 4, gacc + kOffW4, 64, 3, 64);
        back_dense(w.dO, 16, 1, net.W4, 64, 4, w.H3, 64, w.Z0, 64, gacc + kOffB3, nullptr);
        wave_sync();
        // layer 3: dW3 and dZ2
        accum_dw(w.Z0, 64, 4, w.H2, 64, 4, gacc + kOffW3, 64, 64, 64);
        back_dense(w.Z0, 64, 4, net.W3, 64, 4, w.H2, 64, w.Z1, 64, gacc + kOffB2, nullptr);
        wave_sync();
        // layer 2: dW2 and dZ1
        accum_dw(w.Z1, 64, 4, w.H1, 64, 4, gacc + kOffW2, 64, 64, 64);
        back_dense(w.Z1, 64, 4, net.W2, 64, 4, w.H1, 64, w.Z0, 64, gacc + kOffB1, nullptr);
        wave_sync();
        // layer 1: dW1 (64 x 12) and the gradients of the 12 inputs
        accum_dw(w.Z0, 64, 4, w.X0, 32, 1, gacc + kOffW1, 12, 64, 12);
        back_dense(w.Z0, 64, 4, net.W1, 32, 1, nullptr, 0, nullptr, 0, nullptr, w.O);
        wave_sync();
        if (l < 16) {
            if (my_pane >= 0)
                for (int e = 0; e < 8; ++e) atomicAdd(gacc + kOffE + 8 * my_pane + e, w.O[l * 16 + 4 + e]);
        }
        wave_sync();
    }
    for (int off = 32; off > 0; off >>= 1) my_loss += __shfl_xor(my_loss, off);
    if (l == 0) lsum[threadIdx.x >> 6] = my_loss;
    __syncthreads();
    for (int i = threadIdx.x; i < P; i += blockDim.x) partial[(size_t)blockIdx.x * P + i] = gacc[i];
    if (threadIdx.x == 0) loss_partial[blockIdx.x] = lsum[0] + lsum[1] + lsum[2] + lsum[3];
}

// Sum of the block rows into the canonical gradient vector (length P), and of
// the block losses into *loss (the mean loss when inv_n = 1 / m).
__global__ void k_mlp_reduce(int nblk, int P, const float *partial, const float *loss_partial, float inv_n,
                             float *grad, float *loss)
{
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < P; i += gridDim.x * blockDim.x) {
        float s = 0.0f;
        for (int b = 0; b < nblk; ++b) s += partial[(size_t)b * P + i];
        grad[i] = s;
    }
    if (loss && blockIdx.x == 0 && threadIdx.x == 0) {
        float s = 0.0f;
        for (int b = 0; b < nblk; ++b) s += loss_partial[b];
        *loss = s * inv_n;
    }
}

// Adam step on the FP32 master parameters (bias corrections c1 = 1 - b1^t,
// c2 = 1 - b2^t).
__global__ void k_mlp_adam(int P, const float *grad, float *params, float *m1, float *m2, float lr, float b1, float b2,
                           float eps, float c1, float c2)
{
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < P; i += gridDim.x * blockDim.x) {
        const float gi = grad[i];
        const float a = b1 * m1[i] + (1.0f - b1) * gi;
        const float v = b2 * m2[i] + (1.0f - b2) * gi * gi;
        m1[i] = a;
        m2[i] = v;
        params[i] -= lr * (a / c1) / (sqrtf(v / c2) + eps);
    }
}

// Canonical FP32 parameters -> kernel BF16 weights and FP32 biases.
__global__ void k_mlp_pack(const float *p, __bf16 *wb, float *bb)
{
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < kWb + kBb; i += gridDim.x * blockDim.x) {
        if (i < 64 * 32) {
            const int o = i / 32, k = i % 32;
            wb[i] = (__bf16)(k < 12 ? p[kOffW1 + o * 12 + k] : 0.0f);
        } else if (i < 64 * 32 + 4096) {
            wb[i] = (__bf16)p[kOffW2 + (i - 2048)];
        } else if (i < 64 * 32 + 8192) {
            wb[i] = (__bf16)p[kOffW3 + (i - 6144)];
        } else if (i < kWb) {
            const int j = i - 10240, o = j / 64, k = j % 64;
            wb[i] = (__bf16)(o < 3 ? p[kOffW4 + o * 64 + k] : 0.0f);
        } else {
            const int j = i - kWb;
            float v;
            if (j < 64) v = p[kOffB1 + j];
            else if (j < 128) v = p[kOffB2 + j - 64];
            else if (j < 192) v = p[kOffB3 + j - 128];
            else v = (j - 192) < 3 ? p[kOffB4 + j - 192] : 0.0f;
            bb[j] = v;
        }
    }
}

// Inference: (R, T, w) for m tuples.
__global__ void __launch_bounds__(256) k_mlp_infer(uint32_t m, int n_panes, const float *tup, const int32_t *pane,
                                                   const __bf16 *wb, const float *bb, const float *E, float *out,
                                                   int *bad)
{
    __shared__ NetLds net;
    __shared__ WaveBuf wbuf[4];
    load_net(net, wb, bb);
    WaveBuf &w = wbuf[threadIdx.x >> 6];
    const int l = lane_id();
    const uint32_t ntile = (m + 15) / 16;
    const uint32_t wave = (blockIdx.x * blockDim.x + threadIdx.x) >> 6, nw = (gridDim.x * blockDim.x) >> 6;
    for (uint32_t tile = wave; tile < ntile; tile += nw) {
        const uint32_t s0 = tile * 16;
        int my_pane = -1;   // -1: padding or an invalid pane index (reported in *bad)
        if (l < 16) {
            const uint32_t s = s0 + l;
            if (s < m) {
                my_pane = pane[s];
                if ((unsigned)my_pane >= (unsigned)n_panes) {
                    atomicOr(bad, 1);
                    my_pane = -1;
                }
            }
            if (my_pane >= 0) features(tup[4 * s], tup[4 * s + 1], tup[4 * s + 2], tup[4 * s + 3], E + 8 * my_pane,
                                       w.X0 + l * 32);
            else for (int e = 0; e < 32; ++e) w.X0[l * 32 + e] = (__bf16)0.0f;
        }
        wave_sync();
        forward_tile(net, w);
        if (my_pane >= 0) {
            float R, T, wl;
            heads(w.O[l * 16], w.O[l * 16 + 1], w.O[l * 16 + 2], R, T, wl);
            out[3 * (s0 + l)] = R;
            out[3 * (s0 + l) + 1] = T;
            out[3 * (s0 + l) + 2] = wl;
        }
        wave_sync();
    }
}

// Error table of the surrogate: per cell (pane, cos, thickness, density) the
// largest |R - R*| or |T - T*| over the validation tuples in it (atomic max
// on the bits of non-negative floats).  y: network outputs [m][3].
__global__ void k_err_cells(uint32_t m, const float *tup, const int32_t *pane, const float *y, const float *target,
                            int n_panes, int d0, int d1, int d2, uint32_t *table, int *bad)
{
    const int dims[3] = {d0, d1, d2};
    for (uint32_t s = blockIdx.x * blockDim.x + threadIdx.x; s < m; s += gridDim.x * blockDim.x) {
        const int p = pane[s];
        if ((unsigned)p >= (unsigned)n_panes) {
            atomicOr(bad, 1);
            continue;
        }
        const float e = fmaxf(fabsf(y[3 * s] - target[3 * s]), fabsf(y[3 * s + 1] - target[3 * s + 1]));
        const int c = err_cell<float>(dims, p, tup[4 * s], tup[4 * s + 2], tup[4 * s + 3]);
        atomicMax(table + c, __float_as_uint(e));
    }
}

// ---------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------
void launch_mfma_probe(const float *A32, const float *B32, float *C32, const float *A16, const float *B16, float *C16,
                       hipStream_t s)
{
    hipLaunchKernelGGL(k_mfma_probe, dim3(1), dim3(64), 0, s, A32, B32, C32, A16, B16, C16);
}

// FP64 per-tuple sums of the slab Monte Carlo for callers that cannot
// allocate (sdm_slab_mc_noalloc): 4 doubles per tuple, kMcScratchTuples
// tuples (2 MiB per device, held until the process ends).  Host code never
// passes this name to a kernel: it resolves the device address once per
// device (mc_scratch_address) and passes that.
static __device__ __align__(256) double scratch[4 * (size_t)kMcScratchTuples];

int mc_scratch_address(int device, double **out)
{
    static std::mutex mu;
    static double *addr[kMcScratchDevices] = {};
    if (device < 0 || device >= kMcScratchDevices) return -1;
    std::lock_guard<std::mutex> lock(mu);
    if (!addr[device]) {
        // the caller has made `device` current; each device holds its own copy
        void *p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return -1;
        addr[device] = static_cast<double *>(p);
    }
    *out = addr[device];
    return 0;
}

template <class R>
void launch_slab_mc(uint32_t m, uint32_t nph, const float *cos_i, const float *lam, const float *d, const float *rho,
                    const float *n, const float *k, const float *tint, const float *n_ref, double r2_mm,
                    uint64_t seed, uint32_t tuple0, double *acc, float *Rr, float *Tt, float *A, float *W, int num_cu,
                    hipStream_t s)
{
    const size_t n4 = 4 * (size_t)m;
    hipLaunchKernelGGL(k_zero_f64s, dim3((unsigned)std::min<size_t>(4096, (n4 + 255) / 256)), dim3(256), 0, s, acc, n4);
    const uint64_t total = (uint64_t)m * nph;
    const int grid = (int)std::max<uint64_t>(1, std::min<uint64_t>((total + 255) / 256, 16ull * num_cu));
    hipLaunchKernelGGL(k_slab_mc<R>, dim3(grid), dim3(256), 0, s, m, nph, cos_i, lam, d, rho, n, k, tint, n_ref,
                       r2_mm, seed, tuple0, acc);
    hipLaunchKernelGGL(k_slab_mc_out, dim3((unsigned)std::max<uint32_t>(1, std::min<uint32_t>(4096, (m + 255) / 256))),
                       dim3(256), 0, s, m, nph, acc, Rr, Tt, A, W);
}
#define SDM_INST_MC(R)                                                                                              \
    template void launch_slab_mc<R>(uint32_t, uint32_t, const float *, const float *, const float *, const float *, \
                                    const float *, const float *, const float *, const float *, double, uint64_t,  \
                                    uint32_t, double *, float *, float *, float *, float *, int, hipStream_t);
SDM_INST_MC(float)
SDM_INST_MC(double)
#undef SDM_INST_MC

void launch_mlp_pack(const float *params, void *wb, float *bb, hipStream_t s)
{
    hipLaunchKernelGGL(k_mlp_pack, dim3(48), dim3(256), 0, s, params, (__bf16 *)wb, bb);
}

void launch_mlp_grad(uint32_t m, int n_panes, const float *tup, const int32_t *pane, const float *target,
                     const void *wb, const float *bb, const float *E, float inv_n, float *partial, float *loss_partial,
                     int *bad, int nblk, hipStream_t s)
{
    hipLaunchKernelGGL(k_mlp_grad, dim3(nblk), dim3(256), 0, s, m, n_panes, tup, pane, target, (const __bf16 *)wb, bb,
                       E, inv_n, partial, loss_partial, bad);
}

void launch_mlp_reduce(int nblk, int P, const float *partial, const float *loss_partial, float inv_n, float *grad,
                       float *loss, hipStream_t s)
{
    hipLaunchKernelGGL(k_mlp_reduce, dim3(40), dim3(256), 0, s, nblk, P, partial, loss_partial, inv_n, grad, loss);
}

void launch_mlp_adam(int P, const float *grad, float *params, float *m1, float *m2, float lr, float b1, float b2,
                     float eps, float c1, float c2, hipStream_t s)
{
    hipLaunchKernelGGL(k_mlp_adam, dim3(40), dim3(256), 0, s, P, grad, params, m1, m2, lr, b1, b2, eps, c1, c2);
}

void launch_mlp_infer(uint32_t m, int n_panes, const float *tup, const int32_t *pane, const void *wb, const float *bb,
                      const float *E, float *out, int *bad, int num_cu, hipStream_t s)
{
    const int grid = (int)std::max<uint32_t>(1, std::min<uint32_t>((m + 63) / 64, 4u * num_cu));
    hipLaunchKernelGGL(k_mlp_infer, dim3(grid), dim3(256), 0, s, m, n_panes, tup, pane, (const __bf16 *)wb, bb, E, out,
                       bad);
}

__global__ void k_zero_i32(int *p, int n)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0;
}

void launch_zero_i32(int *p, int n, hipStream_t s)
{
    hipLaunchKernelGGL(k_zero_i32, dim3((n + 255) / 256), dim3(256), 0, s, p, n);
}

void launch_err_cells(uint32_t m, const float *tup, const int32_t *pane, const float *y, const float *target,
                      int n_panes, const int dims[3], float *table, int *bad, hipStream_t s)
{
    const int ncell = n_panes * dims[0] * dims[1] * dims[2];
    hipLaunchKernelGGL(k_zero_i32, dim3((ncell + 255) / 256), dim3(256), 0, s, (int *)table, ncell);
    if (m == 0) return;
    const int grid = (int)std::min<uint32_t>(4096, (m + 255) / 256);
    hipLaunchKernelGGL(k_err_cells, dim3(grid), dim3(256), 0, s, m, tup, pane, y, target, n_panes, dims[0], dims[1],
                       dims[2], (uint32_t *)table, bad);
}

int mlp_net_params() { return kNetParams; }
int mlp_wb_elems() { return kWb; }
int mlp_bb_elems() { return kBb; }

}  // namespace sdm
