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

// dH[16][nti*16] = dZ[16][K] W[K][nti*16] with K = 16 * kq (W row-major
// [K][ldw]); then the ReLU mask from Hm (> 0) into Zout (BF16), or, with
// dx_out, the raw products (FP32, 16 columns) for the input gradients.
__device__ __forceinline__ void back_dense(const __bf16 *dZ, int ldz, int kq, const __bf16 *W, int ldw, int nti,
                                           const __bf16 *Hm, int ldm, __bf16 *Zout, int ldo, float *dx_out)
{
    const int l = lane_id(), g = l / 16, c = l % 16;
    for (int ti = 0; ti < nti; ++ti) {
        f32x4 acc = {0, 0, 0, 0};
        for (int kk = 0; kk < kq; ++kk) {
            // dZ[c][16 kk + 4 g .. + 3]: one 8-byte read (row strides are multiples of 8 bytes)
            const s16x4 a = *reinterpret_cast<const s16x4 *>(dZ + c * ldz + 16 * kk + 4 * g);
            s16x4 bv;
            for (int j = 0; j < 4; ++j) bv[j] = bits(W[(16 * kk + 4 * g + j) * ldw + 16 * ti + c]);
            acc = mfma16(a, bv, acc);
        }
        for (int r = 0; r < 4; ++r) {
            const int s = 4 * g + r, i = 16 * ti + c;
            if (dx_out) {
                dx_out[s * 16 + c] = acc[r];
                continue;
            }
            Zout[s * ldo + i] = (__bf16)((float)Hm[s * ldm + i] > 0.0f ? acc[r] : 0.0f);
        }
    }
}

// One 16x16 tile of a block's weight gradient dW[out][in] = sum over the
// block's 64 samples of dZ[s][out] H[s][in]: the samples are the products'
// K dimension, 16 from each wave's buffers (wave q's at A0 + q * as and
// B0 + q * bs), chained into the accumulator.
__device__ __forceinline__ f32x4 dw_tile(f32x4 acc, const __bf16 *A0, int lda, int as, int to, const __bf16 *B0,
                                        int ldb, int bs, int ti)
{
    const int l = lane_id(), g = l / 16, c = l % 16;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const __bf16 *A = A0 + q * as, *B = B0 + q * bs;
        s16x4 a, bv;
        for (int j = 0; j < 4; ++j) {
            a[j] = bits(A[(4 * g + j) * lda + 16 * to + c]);
            bv[j] = bits(B[(4 * g + j) * ldb + 16 * ti + c]);
        }
        acc = mfma16(a, bv, acc);
    }
    return acc;
}

// The 40 weight-gradient tiles of the network: W4 (3 x 64, one padded row
// tile), W3 and W2 (16 tiles each), W1 (64 x 12, one padded column tile).
struct DwTile {
    int layer, to, ti;
};
__device__ __forceinline__ DwTile dw_tile_of(int k)
{
    if (k < 4) return {4, 0, k};
    if (k < 20) return {3, (k - 4) / 4, (k - 4) % 4};
    if (k < 36) return {2, (k - 20) / 4, (k - 20) % 4};
    return {1, k - 36, 0};
}

// Gradient of the mean loss over a batch of m samples (inv_n = 1 / m).  A
// block takes groups of 64 samples, one 16-sample tile per wave: each wave
// runs its tile forward and backward and leaves every layer's dZ and input
// in LDS; the block then forms the weight gradients as matrix-core products
// over the 64 samples (ten tiles per wave, accumulated in registers over all
// the block's groups), and bias, embedding and loss sums in a fixed order.
// Each block writes one row of P = 9347 + 8 n_panes values once, with no
// atomics, so the gradient does not depend on scheduling.
__global__ void __launch_bounds__(256) k_mlp_grad(uint32_t m, int n_panes, const float *tup, const int32_t *pane,
                                                  const float *target, const __bf16 *wb, const float *bb,
                                                  const float *E, float inv_n, float *partial, float *loss_partial,
                                                  int *bad)
{
    __shared__ NetLds net;
    __shared__ WaveBuf wbuf[4];
    __shared__ __bf16 zd1[4][16 * kLd64];   // dZ of layer 1, per wave
    __shared__ float gO[4][16 * 4];       // d loss / d o of each sample (FP32)
    __shared__ int32_t spane[64];         // pane of each sample of the group (-1: none)
    __shared__ float lsum[4];
    const int P = kNetParams + 8 * n_panes;
    const int wv = threadIdx.x >> 6, l = lane_id(), t = threadIdx.x;
    const uint32_t ngrp = (m + 63) / 64;
    // this lane's sample of a group (lanes 0-15): pane, inputs and target,
    // fetched ahead of use (the first group's before the weights are staged)
    int my_pane = -1;
    bool have = false;   // the lane has a sample (not padding)
    float fin[4] = {0, 0, 0, 0}, tg[3] = {0, 0, 0};
    auto fetch = [&](uint32_t grp) {
        const uint32_t s = grp * 64 + 16 * wv + l;
        have = l < 16 && grp < ngrp && s < m;
        if (have) {
            my_pane = pane[s];
            for (int q = 0; q < 4; ++q) fin[q] = tup[4 * s + q];
            for (int q = 0; q < 3; ++q) tg[q] = target[3 * s + q];
        }
    };
    fetch(blockIdx.x);
    load_net(net, wb, bb);
    WaveBuf &w = wbuf[wv];
    const int ws = (int)(sizeof(WaveBuf) / sizeof(__bf16));
    f32x4 acc[10];
#pragma unroll
    for (int u = 0; u < 10; ++u) acc[u] = f32x4{0, 0, 0, 0};
    float bsum = 0.0f, esum0 = 0.0f, esum1 = 0.0f, my_loss = 0.0f;
    const int pe0 = t, pe1 = t + 256;   // (pane, embedding) pairs of this thread: p = pe / 8, e = pe % 8
    for (uint32_t grp = blockIdx.x; grp < ngrp; grp += gridDim.x) {
        // -1: padding or an invalid pane index (reported in *bad)
        if (!have) my_pane = -1;
        else if ((unsigned)my_pane >= (unsigned)n_panes) {
            atomicOr(bad, 1);
            my_pane = -1;
        }
        if (l < 16) {
            if (my_pane >= 0) features(fin[0], fin[1], fin[2], fin[3], E + 8 * my_pane, w.X0 + l * kLd32);
            else for (int e = 0; e < 32; ++e) w.X0[l * kLd32 + e] = (__bf16)0.0f;
            spane[16 * wv + l] = my_pane;
        }
        wave_sync();
        forward_tile(net, w);
        // heads, loss and d loss / d o; padded samples get a zero gradient
        if (l < 16) {
            float go0 = 0, go1 = 0, go2 = 0;
            if (my_pane >= 0) {
                const float o0 = w.O[l * 16], o1 = w.O[l * 16 + 1], o2 = w.O[l * 16 + 2];
                float R, T, wl;
                heads(o0, o1, o2, R, T, wl);
                const float e0 = R - tg[0], e1 = T - tg[1], e2 = wl - tg[2];
                my_loss += e0 * e0 + e1 * e1 + e2 * e2;
                const float gR = 2.0f * e0 * inv_n, gT = 2.0f * e1 * inv_n, gw = 2.0f * e2 * inv_n;
                go0 = gR * R * (1.0f - R) - gT * T * R;
                go1 = -gR * R * T + gT * T * (1.0f - T);
                go2 = gw / (1.0f + expf(-o2));
            }
            gO[wv][l * 4] = go0;
            gO[wv][l * 4 + 1] = go1;
            gO[wv][l * 4 + 2] = go2;
            for (int q = 0; q < 16; ++q)
                w.dO[l * kLd16 + q] = (__bf16)(q == 0 ? go0 : q == 1 ? go1 : q == 2 ? go2 : 0.0f);
        }
        wave_sync();
        // dZ3 = (dO W4) masked by H3, dZ2, dZ1, then the inputs' gradients
        back_dense(w.dO, kLd16, 1, net.W4, kLd64, 4, w.H3, kLd64, w.Z0, kLd64, nullptr);
        wave_sync();
        back_dense(w.Z0, kLd64, 4, net.W3, kLd64, 4, w.H2, kLd64, w.Z1, kLd64, nullptr);
        wave_sync();
        back_dense(w.Z1, kLd64, 4, net.W2, kLd64, 4, w.H1, kLd64, zd1[wv], kLd64, nullptr);
        wave_sync();
        back_dense(zd1[wv], kLd64, 4, net.W1, kLd32, 1, nullptr, 0, nullptr, 0, w.O);
        fetch(grp + gridDim.x);   // the next group's samples, while the block finishes this one
        __syncthreads();
        // weight gradients over the group's 64 samples: tiles wv, wv + 4, ...
#pragma unroll
        for (int u = 0; u < 10; ++u) {
            const DwTile d = dw_tile_of(wv + 4 * u);
            if (d.layer == 4) acc[u] = dw_tile(acc[u], wbuf[0].dO, kLd16, ws, d.to, wbuf[0].H3, kLd64, ws, d.ti);
            else if (d.layer == 3) acc[u] = dw_tile(acc[u], wbuf[0].Z0, kLd64, ws, d.to, wbuf[0].H2, kLd64, ws, d.ti);
            else if (d.layer == 2) acc[u] = dw_tile(acc[u], wbuf[0].Z1, kLd64, ws, d.to, wbuf[0].H1, kLd64, ws, d.ti);
            else acc[u] = dw_tile(acc[u], zd1[0], kLd64, 16 * kLd64, d.to, wbuf[0].X0, kLd32, ws, d.ti);
        }
        // bias sums: threads 0-63 layer 1, 64-127 layer 2, 128-191 layer 3, 192-194 the outputs
        if (t < 192) {
            const int col = t & 63;
            for (int q = 0; q < 4; ++q)
                for (int r = 0; r < 16; ++r) {
                    const __bf16 *D = t < 64 ? zd1[q] : (t < 128 ? wbuf[q].Z1 : wbuf[q].Z0);
                    bsum += (float)D[r * kLd64 + col];
                }
        } else if (t < 195) {
            for (int q = 0; q < 4; ++q)
                for (int r = 0; r < 16; ++r) bsum += gO[q][r * 4 + (t - 192)];
        }
        // embedding rows: the inputs' gradients 4..11 of the samples of each pane
        if (pe0 < 8 * n_panes)
            for (int s = 0; s < 64; ++s)
                if (spane[s] == pe0 / 8) esum0 += wbuf[s / 16].O[(s % 16) * 16 + 4 + pe0 % 8];
        if (pe1 < 8 * n_panes)
            for (int s = 0; s < 64; ++s)
                if (spane[s] == pe1 / 8) esum1 += wbuf[s / 16].O[(s % 16) * 16 + 4 + pe1 % 8];
        __syncthreads();
    }
    float *row = partial + (size_t)blockIdx.x * P;
    const int g = l / 16, c = l % 16;
#pragma unroll
    for (int u = 0; u < 10; ++u) {
        const DwTile d = dw_tile_of(wv + 4 * u);
        const int off = d.layer == 4 ? kOffW4 : d.layer == 3 ? kOffW3 : d.layer == 2 ? kOffW2 : kOffW1;
        const int ldd = d.layer == 1 ? 12 : 64, out_max = d.layer == 4 ? 3 : 64, in_max = d.layer == 1 ? 12 : 64;
        for (int r = 0; r < 4; ++r) {
            const int o = 16 * d.to + 4 * g + r, i = 16 * d.ti + c;
            if (o < out_max && i < in_max) row[off + o * ldd + i] = acc[u][r];
        }
    }
    if (t < 64) row[kOffB1 + t] = bsum;
    else if (t < 128) row[kOffB2 + t - 64] = bsum;
    else if (t < 192) row[kOffB3 + t - 128] = bsum;
    else if (t < 195) row[kOffB4 + t - 192] = bsum;
    if (pe0 < 8 * n_panes) row[kOffE + pe0] = esum0;
    if (pe1 < 8 * n_panes) row[kOffE + pe1] = esum1;
    for (int off = 32; off > 0; off >>= 1) my_loss += __shfl_xor(my_loss, off);
    if (l == 0) lsum[wv] = my_loss;
    __syncthreads();
    if (t == 0) loss_partial[blockIdx.x] = (lsum[0] + lsum[1]) + (lsum[2] + lsum[3]);
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

// Where canonical parameter i lives in the kernels' layout: the BF16 weight
// index (*is_w = true) or the FP32 bias index; -1 for the embedding, which
// the kernels read from the FP32 parameters.
__device__ __forceinline__ int packed_index(int i, bool *is_w)
{
    *is_w = true;
    if (i < kOffB1) return (i / 12) * 32 + i % 12;
    if (i < kOffW2) { *is_w = false; return i - kOffB1; }
    if (i < kOffB2) return 2048 + (i - kOffW2);
    if (i < kOffW3) { *is_w = false; return 64 + (i - kOffB2); }
    if (i < kOffB3) return 6144 + (i - kOffW3);
    if (i < kOffW4) { *is_w = false; return 128 + (i - kOffB3); }
    if (i < kOffB4) return 10240 + i - kOffW4;   // W4 rows 0..2 of the 16-row padded block
    if (i < kOffE) { *is_w = false; return 192 + (i - kOffB4); }
    return -1;
}

// One training step after the gradient pass: the block rows summed in a fixed
// order (eight interleaved partial sums per parameter, combined pairwise),
// the Adam step on the FP32 master parameters (bias corrections c1 = 1 - b1^t,
// c2 = 1 - b2^t), and the new parameters' BF16 / FP32 copies that the next
// gradient pass reads.  Block 0 also writes the mean loss.
constexpr int kRaPar = 32;   // parameters per block, 8 threads each
__global__ void __launch_bounds__(256) k_mlp_reduce_adam(int nblk, int P, const float *partial,
                                                         const float *loss_partial, float inv_n, float *loss,
                                                         float *params, float *m1, float *m2, float lr, float b1,
                                                         float b2, float eps, float c1, float c2, __bf16 *wb,
                                                         float *bb)
{
    __shared__ float s[8][kRaPar];
    const int c = threadIdx.x % kRaPar, q = threadIdx.x / kRaPar;
    const int i = blockIdx.x * kRaPar + c;
    float sum = 0.0f;
    if (i < P) {
        // rows q, q + 8, q + 16, ... in order; eight loads in flight per round
        const float *col = partial + i;
        int b = q;
        for (; b + 56 < nblk; b += 64) {
            float v[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) v[u] = col[(size_t)(b + 8 * u) * P];
#pragma unroll
            for (int u = 0; u < 8; ++u) sum += v[u];
        }
        for (; b < nblk; b += 8) sum += col[(size_t)b * P];
    }
    // the state the update needs, loaded while the sums complete
    float m1i = 0.0f, m2i = 0.0f, pi = 0.0f;
    if (q == 0 && i < P) {
        m1i = m1[i];
        m2i = m2[i];
        pi = params[i];
    }
    s[q][c] = sum;
    __syncthreads();
    if (q == 0 && i < P) {
        const float gi = ((s[0][c] + s[1][c]) + (s[2][c] + s[3][c])) + ((s[4][c] + s[5][c]) + (s[6][c] + s[7][c]));
        const float a = b1 * m1i + (1.0f - b1) * gi;
        const float v = b2 * m2i + (1.0f - b2) * gi * gi;
        m1[i] = a;
        m2[i] = v;
        const float p = pi - lr * (a / c1) / (sqrtf(v / c2) + eps);
        params[i] = p;
        bool is_w;
        const int k = packed_index(i, &is_w);
        if (k >= 0) {
            if (is_w) wb[k] = (__bf16)p;
            else bb[k] = p;
        }
    }
    if (loss && blockIdx.x == 0 && threadIdx.x >= 64 && threadIdx.x < 128) {
        // the block losses over one wave: lane l sums l, l + 64, ...; then a
        // fixed butterfly
        const int ln = threadIdx.x - 64;
        float t = 0.0f;
        for (int b = ln; b < nblk; b += 64) t += loss_partial[b];
        for (int off = 32; off > 0; off >>= 1) t += __shfl_xor(t, off);
        if (ln == 0) *loss = t * inv_n;
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
                                       w.X0 + l * kLd32);
            else for (int e = 0; e < 32; ++e) w.X0[l * kLd32 + e] = (__bf16)0.0f;
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

void launch_mlp_reduce_adam(int nblk, int P, const float *partial, const float *loss_partial, float inv_n, float *loss,
                            float *params, float *m1, float *m2, float lr, float b1, float b2, float eps, float c1,
                            float c2, void *wb, float *bb, hipStream_t s)
{
    hipLaunchKernelGGL(k_mlp_reduce_adam, dim3((P + kRaPar - 1) / kRaPar), dim3(256), 0, s, nblk, P, partial,
                       loss_partial, inv_n, loss, params, m1, m2, lr, b1, b2, eps, c1, c2, (__bf16 *)wb, bb);
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
