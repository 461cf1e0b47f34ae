// sr_mlp.hip -- the MLP surrogate of the inverse number-CDF: inference,
// training (mean-squared error on log2 x, gradients on the matrix cores), Adam,
// and the generation of training triples from the FP64-built tables.
#include <math.h>

#include <algorithm>

#include "sr_mlp.hpp"

namespace sr {
namespace {

// ------------------------------------------------------------------ inference
__global__ __launch_bounds__(kBlock) void mlp_forward_kernel(const __bf16 *__restrict__ params,
                                                             const float2 *__restrict__ feats,
                                                             float *__restrict__ out, int64_t M) {
    __shared__ MlpSmem s;
    __shared__ alignas(16) __bf16 tbuf[kWaves][2 * 16 * kH];
    mlp_load(s, params, threadIdx.x, blockDim.x);
    __syncthreads();
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63, r = lane & 15;
    for (int64_t tile = (int64_t)blockIdx.x * kWaves + wave; tile * 16 < M;
         tile += (int64_t)gridDim.x * kWaves) {
        const int64_t idx = tile * 16 + r;
        const bool valid = idx < M;
        const float2 f = valid ? feats[idx] : make_float2(0.f, 0.f);
        const float y = mlp_tile16(s, tbuf[wave], f.x, f.y);
        if (valid && lane < 16) out[idx] = y;
    }
}

// ------------------------------------------------------------------ training
__device__ __forceinline__ float dsilu(float z) {
    const float sg = __builtin_amdgcn_rcpf(1.0f + __expf(-z));
    return sg * (1.0f + z * (1.0f - sg));
}

struct alignas(16) TrainSmem {
    MlpSmem m;
    alignas(16) __bf16 W2T[kH * kH];   // W2T[k][j] = W2[j][k]
    alignas(16) __bf16 W3T[kH * kH];
};

// Gradient of L = (1/M) sum w (y - t)^2, w = x / E[x] (the energy weighting of
// the binned spectrum the network is judged on), for this kernel's tiles; with
// VJP, the gradient of sum dout * y instead (`target` holds dout, inv_m unused).
// Each wave accumulates its own gradient and writes it to work[wave_global][...]
// (summed in a fixed order by grad_reduce).
template <bool VJP>
__global__ __launch_bounds__(kBlock) void mlp_train_kernel(const __bf16 *__restrict__ params,
                                                           const float2 *__restrict__ feats,
                                                           const float *__restrict__ target,
                                                           int64_t M, float inv_m,
                                                           float *__restrict__ work) {
    __shared__ TrainSmem s;
    __shared__ alignas(16) __bf16 tbuf[kWaves][2 * 16 * kH];
    mlp_load(s.m, params, threadIdx.x, blockDim.x);
    for (int i = threadIdx.x; i < kH * kH; i += blockDim.x) {
        const int j = i / kH, k = i % kH;
        s.W2T[k * kH + j] = params[kOffW2 + i];
        s.W3T[k * kH + j] = params[kOffW3 + i];
    }
    __syncthreads();
    const int wave = threadIdx.x >> 6, l = threadIdx.x & 63, r = l & 15, g = l >> 4;
    __bf16 *tb = tbuf[wave];

    f32x4 gW2[4][4], gW3[4][4];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            gW2[a][b] = (f32x4){0.f, 0.f, 0.f, 0.f};
            gW3[a][b] = (f32x4){0.f, 0.f, 0.f, 0.f};
        }
    float gW1[4][2], gb1[4], gb2[4], gb3[4], gW4[4], gb4 = 0.f;
#pragma unroll
    for (int n = 0; n < 4; ++n) {
        gW1[n][0] = gW1[n][1] = gb1[n] = gb2[n] = gb3[n] = gW4[n] = 0.f;
    }

    for (int64_t tile = (int64_t)blockIdx.x * kWaves + wave; tile * 16 < M;
         tile += (int64_t)gridDim.x * kWaves) {
        const int64_t idx = tile * 16 + r;
        const bool valid = idx < M;
        const float2 f = valid ? feats[idx] : make_float2(0.f, 0.f);
        const float tgt = valid ? target[idx] : 0.f;
        // features of the samples of the D-layout rows 4g+q
        float fq0[4], fq1[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            fq0[q] = __shfl(f.x, 4 * g + q, 64);
            fq1[q] = __shfl(f.y, 4 * g + q, 64);
        }
        // ---- forward, keeping pre-activations in the D layout
        Split8 a[2];
#pragma unroll
        for (int kb = 0; kb < 2; ++kb)
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                const int k = 32 * kb + 8 * g + e;
                split_set(a[kb], e, silu(fmaf(s.m.W1[2 * k], f.x, fmaf(s.m.W1[2 * k + 1], f.y, s.m.b1[k]))));
            }
        float z1[4][4];   // z1[n][q]: sample 4g+q, feature 16n+r
#pragma unroll
        for (int n = 0; n < 4; ++n) {
            const int k = 16 * n + r;
#pragma unroll
            for (int q = 0; q < 4; ++q)
                z1[n][q] = fmaf(s.m.W1[2 * k], fq0[q], fmaf(s.m.W1[2 * k + 1], fq1[q], s.m.b1[k]));
        }
        f32x4 z2[4];
#pragma unroll
        for (int n = 0; n < 4; ++n) {
            z2[n] = (f32x4){0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int kb = 0; kb < 2; ++kb) {
                const bf16x8 b = *(const bf16x8 *)&s.m.W2[(16 * n + r) * kH + 32 * kb + 8 * g];
                z2[n] = mfma_split(a[kb], b, z2[n]);
            }
#pragma unroll
            for (int q = 0; q < 4; ++q) z2[n][q] += s.m.b2[16 * n + r];
        }
#pragma unroll
        for (int n = 0; n < 4; ++n)
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const float v = silu(z2[n][q]);
                const __bf16 h = (__bf16)v;
                tb[(4 * g + q) * kH + 16 * n + r] = h;
                tb[16 * kH + (4 * g + q) * kH + 16 * n + r] = (__bf16)(v - (float)h);
            }
        wave_lds_sync();
#pragma unroll
        for (int kb = 0; kb < 2; ++kb) {
            a[kb].hi = *(const bf16x8 *)&tb[r * kH + 32 * kb + 8 * g];
            a[kb].lo = *(const bf16x8 *)&tb[16 * kH + r * kH + 32 * kb + 8 * g];
        }
        wave_lds_sync();
        f32x4 z3[4];
#pragma unroll
        for (int n = 0; n < 4; ++n) {
            z3[n] = (f32x4){0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int kb = 0; kb < 2; ++kb) {
                const bf16x8 b = *(const bf16x8 *)&s.m.W3[(16 * n + r) * kH + 32 * kb + 8 * g];
                z3[n] = mfma_split(a[kb], b, z3[n]);
            }
#pragma unroll
            for (int q = 0; q < 4; ++q) z3[n][q] += s.m.b3[16 * n + r];
        }
        float sq[4] = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int n = 0; n < 4; ++n)
#pragma unroll
            for (int q = 0; q < 4; ++q) sq[q] = fmaf(s.m.W4[16 * n + r], silu(z3[n][q]), sq[q]);
#pragma unroll
        for (int q = 0; q < 4; ++q)
#pragma unroll
            for (int o = 8; o > 0; o >>= 1) sq[q] += __shfl_xor(sq[q], o, 64);
        // dL/dy of the rows 4g+q (zero for padding samples)
        float dyq[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const float tq = __shfl(tgt, 4 * g + q, 64);
            const bool vq = tile * 16 + 4 * g + q < M;
            if constexpr (VJP) {
                dyq[q] = vq ? tq : 0.f;
            } else {
                // energy weighting: each sample counts with x / E[x] (E[x] = 8/(15 sqrt3) ...)
                const float wq = exp2f(tq) * 3.2475953f;
                dyq[q] = vq ? 2.0f * inv_m * wq * (sq[q] + s.m.b4 - tq) : 0.f;
            }
        }
        if (r == 0) gb4 += dyq[0] + dyq[1] + dyq[2] + dyq[3];
        // ---- layer 4 and 3
        f32x4 dz3[4];
#pragma unroll
        for (int n = 0; n < 4; ++n) {
            const float w4 = s.m.W4[16 * n + r];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                gW4[n] = fmaf(dyq[q], silu(z3[n][q]), gW4[n]);
                dz3[n][q] = dyq[q] * w4 * dsilu(z3[n][q]);
                gb3[n] += dz3[n][q];
            }
        }
        // h2 in the D layout (the B operand of dW3 = dZ3^T H2)
        bf16x4 h2b[4], dz3b[4];
#pragma unroll
        for (int n = 0; n < 4; ++n)
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                h2b[n][q] = (__bf16)silu(z2[n][q]);
                dz3b[n][q] = (__bf16)dz3[n][q];
            }
#pragma unroll
        for (int nj = 0; nj < 4; ++nj)
#pragma unroll
            for (int nk = 0; nk < 4; ++nk)
                gW3[nj][nk] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(dz3b[nj], h2b[nk], gW3[nj][nk], 0, 0, 0);
        // dh2 = dZ3 W3: dZ3 to the A layout through LDS, B from W3T
#pragma unroll
        for (int n = 0; n < 4; ++n)
#pragma unroll
            for (int q = 0; q < 4; ++q) tb[(4 * g + q) * kH + 16 * n + r] = dz3b[n][q];
        wave_lds_sync();
#pragma unroll
        for (int kb = 0; kb < 2; ++kb) a[kb].hi = *(const bf16x8 *)&tb[r * kH + 32 * kb + 8 * g];
        wave_lds_sync();
        f32x4 dz2[4];
#pragma unroll
        for (int n = 0; n < 4; ++n) {
            dz2[n] = (f32x4){0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int kb = 0; kb < 2; ++kb) {
                const bf16x8 b = *(const bf16x8 *)&s.W3T[(16 * n + r) * kH + 32 * kb + 8 * g];
                dz2[n] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[kb].hi, b, dz2[n], 0, 0, 0);
            }
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                dz2[n][q] *= dsilu(z2[n][q]);
                gb2[n] += dz2[n][q];
            }
        }
        // dW2 = dZ2^T H1 with H1 in the D layout
        bf16x4 h1b[4], dz2b[4];
#pragma unroll
        for (int n = 0; n < 4; ++n)
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                h1b[n][q] = (__bf16)silu(z1[n][q]);
                dz2b[n][q] = (__bf16)dz2[n][q];
            }
#pragma unroll
        for (int nj = 0; nj < 4; ++nj)
#pragma unroll
            for (int nk = 0; nk < 4; ++nk)
                gW2[nj][nk] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(dz2b[nj], h1b[nk], gW2[nj][nk], 0, 0, 0);
        // dh1 = dZ2 W2
#pragma unroll
        for (int n = 0; n < 4; ++n)
#pragma unroll
            for (int q = 0; q < 4; ++q) tb[(4 * g + q) * kH + 16 * n + r] = dz2b[n][q];
        wave_lds_sync();
#pragma unroll
        for (int kb = 0; kb < 2; ++kb) a[kb].hi = *(const bf16x8 *)&tb[r * kH + 32 * kb + 8 * g];
        wave_lds_sync();
#pragma unroll
        for (int n = 0; n < 4; ++n) {
            f32x4 dh1 = (f32x4){0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int kb = 0; kb < 2; ++kb) {
                const bf16x8 b = *(const bf16x8 *)&s.W2T[(16 * n + r) * kH + 32 * kb + 8 * g];
                dh1 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[kb].hi, b, dh1, 0, 0, 0);
            }
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const float dz1 = dh1[q] * dsilu(z1[n][q]);
                gb1[n] += dz1;
                gW1[n][0] = fmaf(dz1, fq0[q], gW1[n][0]);
                gW1[n][1] = fmaf(dz1, fq1[q], gW1[n][1]);
            }
        }
    }

    // ---- this wave's gradient -> work[wave_global][kNParams]
    float *out = work + ((int64_t)blockIdx.x * kWaves + wave) * kNParams;
#pragma unroll
    for (int n = 0; n < 4; ++n) {
        float v[6] = {gW1[n][0], gW1[n][1], gb1[n], gb2[n], gb3[n], gW4[n]};
#pragma unroll
        for (int c = 0; c < 6; ++c) {
            v[c] += __shfl_xor(v[c], 16, 64);
            v[c] += __shfl_xor(v[c], 32, 64);
        }
        if (g == 0) {
            const int j = 16 * n + r;
            out[kOffW1 + 2 * j] = v[0];
            out[kOffW1 + 2 * j + 1] = v[1];
            out[kOffB1 + j] = v[2];
            out[kOffB2 + j] = v[3];
            out[kOffB3 + j] = v[4];
            out[kOffW4 + j] = v[5];
        }
    }
    float b4 = gb4;
    b4 += __shfl_xor(b4, 16, 64);
    b4 += __shfl_xor(b4, 32, 64);
    if (l == 0) out[kOffB4] = b4;
#pragma unroll
    for (int nj = 0; nj < 4; ++nj)
#pragma unroll
        for (int nk = 0; nk < 4; ++nk)
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int j = 16 * nj + 4 * g + q, k = 16 * nk + r;
                out[kOffW2 + j * kH + k] = gW2[nj][nk][q];
                out[kOffW3 + j * kH + k] = gW3[nj][nk][q];
            }
}

// grads[p] = sum over waves of work[wave][p] (fixed order).
// Sum of the per-wave gradient rows, in two fixed-order stages: blockIdx.y
// sums rows [y * per, (y + 1) * per) into out row y.
__global__ void grad_reduce_kernel(const float *__restrict__ work, int nrows, int per,
                                   float *__restrict__ out) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= kNParams) return;
    const int r0 = blockIdx.y * per, r1 = min(r0 + per, nrows);
    float sum = 0.f;
#pragma unroll 8
    for (int w = r0; w < r1; ++w) sum += work[(int64_t)w * kNParams + p];
    out[(int64_t)blockIdx.y * kNParams + p] = sum;
}

__global__ void adam_kernel(float *__restrict__ master, __bf16 *__restrict__ params,
                            const float *__restrict__ grads, float *__restrict__ m,
                            float *__restrict__ v, float lr, float b1, float b2, float eps,
                            float c1, float c2) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= kNParams) return;
    const float gr = grads[p];
    const float mm = b1 * m[p] + (1.f - b1) * gr;
    const float vv = b2 * v[p] + (1.f - b2) * gr * gr;
    m[p] = mm;
    v[p] = vv;
    const float w = master[p] - lr * (mm * c1) / (sqrtf(vv * c2) + eps);
    master[p] = w;
    params[p] = (__bf16)w;
}

__global__ void cast_kernel(const float *__restrict__ master, __bf16 *__restrict__ params) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p < kNParams) params[p] = (__bf16)master[p];
}

// Training triples: log10 chi uniform on [lo, hi], u a 23-bit midpoint, target
// log2 x from the tables (x = T1(u r(chi)), r = 1 without the cut), clipped
// below at x = 1e-5 where photons carry no measurable energy.
__global__ void make_batch_kernel(TableDev tab, uint32_t k0, uint32_t k1, uint32_t batch,
                                  int kin_cut, float lo, float hi, float2 *__restrict__ feats,
                                  float *__restrict__ target, int64_t M) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= M) return;
    const uint4 w = philox4x32_10(make_uint4((uint32_t)i, (uint32_t)(i >> 32), batch, 3u), k0, k1);
    const float lchi = lo + (hi - lo) * ((float)(w.x >> 8) * 0x1p-24f);
    const float chi = exp2f(lchi * 3.3219280948873623f);
    const float2 rr = kin_cut ? r_lookup(tab.r, chi) : make_float2(1.0f, 0.0f);
    float lnU, ln1mU;
    direct_u(w.y, rr, lnU, ln1mU);
    const float y = fmaxf(t1_log2x(tab.t1, lnU, ln1mU), kMlpLog2xFloor);
    feats[i] = make_float2((lchi + 1.0f) * (1.0f / 3.0f), mlp_feature_u(w.y));
    target[i] = y;
}

__global__ void eval_direct_kernel(TableDev tab, const uint32_t *__restrict__ a,
                                   const float *__restrict__ chi, int kin_cut,
                                   float *__restrict__ out, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float2 rr = kin_cut ? r_lookup(tab.r, chi[i]) : make_float2(1.0f, 0.0f);
    float lnU, ln1mU;
    direct_u(a[i], rr, lnU, ln1mU);
    out[i] = exp2f(t1_log2x(tab.t1, lnU, ln1mU));
}

constexpr int kTrainBlocks = 256;      // one block (four waves, one per SIMD) per CU
constexpr int kGradGroups = 32;        // first-stage row groups of the gradient sum

// ------------------------------------------------------------------ the judge
// Sample s of the judge's stratified grid: chi-bin b (of kMlpFallbackBins on
// log10 chi in [kMlpChiLo, kMlpChiHi)), chi value j of cpb at the centres of b's
// sub-intervals, u the m-th of n_u 23-bit midpoints spread evenly over (0, 1).
struct JudgeGrid {
    int n_u, cpb;
    float width;        // log10 chi per bin
};
__device__ __forceinline__ void judge_sample(const JudgeGrid &G, int64_t s, float &lchi, float &chi,
                                             uint32_t &word) {
    const int64_t per_bin = (int64_t)G.cpb * G.n_u;
    const int b = (int)(s / per_bin);
    const int j = (int)((s / G.n_u) % G.cpb);
    const int m = (int)(s % G.n_u);
    lchi = kMlpChiLo + G.width * ((float)b + ((float)j + 0.5f) / (float)G.cpb);
    chi = exp2f(lchi * 3.3219280948873623f);
    const uint32_t mu = (uint32_t)(((double)m + 0.5) * (8388608.0 / (double)G.n_u));
    word = mu << 9;
}

// x from the table sampler and the network's features of every judge sample.
__global__ void judge_inputs_kernel(TableDev tab, JudgeGrid G, int kin_cut, int64_t total,
                                    float *__restrict__ x_tab, float2 *__restrict__ feats) {
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= total) return;
    float lchi, chi;
    uint32_t word;
    judge_sample(G, s, lchi, chi, word);
    const float2 rr = kin_cut ? r_lookup(tab.r, chi) : make_float2(1.0f, 0.0f);
    float lnU, ln1mU;
    direct_u(word, rr, lnU, ln1mU);
    x_tab[s] = exp2f(t1_log2x(tab.t1, lnU, ln1mU));
    feats[s] = make_float2((lchi + 1.0f) * (1.0f / 3.0f), mlp_feature_u(word));
}

// Energy-weighted histograms of the two samplers' x over n_xb log bins of
// [x_lo, x_hi): block (b, part) adds the samples of chi-bin b in its share to
// hist[b][0][.] (table) and hist[b][1][.] (network) (FP64).
__global__ __launch_bounds__(256) void judge_hist_kernel(JudgeGrid G, const float *__restrict__ x_tab,
                                                         const float *__restrict__ y_net,
                                                         double l_lo, double inv_w, int n_xb,
                                                         double *__restrict__ hist) {
    extern __shared__ double sh[];   // [2 * n_xb]
    for (int i = threadIdx.x; i < 2 * n_xb; i += blockDim.x) sh[i] = 0.0;
    __syncthreads();
    const int b = blockIdx.y;
    const int64_t per_bin = (int64_t)G.cpb * G.n_u;
    const int64_t s0 = (int64_t)b * per_bin;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < per_bin;
         i += (int64_t)gridDim.x * blockDim.x) {
        const double xs[2] = {(double)x_tab[s0 + i], (double)exp2f(y_net[s0 + i])};
#pragma unroll
        for (int v = 0; v < 2; ++v) {
            const double x = xs[v];
            if (!(x > 0.0)) continue;
            const double u = (log(x) - l_lo) * inv_w;
            if (u >= 0.0 && u < (double)n_xb) atomicAdd(&sh[v * n_xb + (int)u], x);
        }
    }
    __syncthreads();
    for (int i = threadIdx.x; i < 2 * n_xb; i += blockDim.x)
        if (sh[i] != 0.0) atomicAdd(&hist[(int64_t)b * 2 * n_xb + i], sh[i]);
}

// err[b] = sum |h_net - h_tab| / sum h_tab; fallback[b] = err[b] > tol.
__global__ void judge_err_kernel(const double *__restrict__ hist, int n_xb, double tol,
                                 double *__restrict__ err, uint8_t *__restrict__ fallback) {
    const int b = blockIdx.x;
    double d = 0.0, t = 0.0;
    for (int i = threadIdx.x; i < n_xb; i += 64) {
        const double ht = hist[(int64_t)b * 2 * n_xb + i];
        const double hn = hist[(int64_t)b * 2 * n_xb + n_xb + i];
        d += fabs(hn - ht);
        t += ht;
    }
    d = wave_sum(d);
    t = wave_sum(t);
    if (threadIdx.x == 0) {
        const double e = d / fmax(t, 1e-300);
        err[b] = e;
        fallback[b] = (uint8_t)(!(e <= tol));
    }
}

__global__ void zero_doubles_kernel(double *__restrict__ p, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0.0;
}

int launch_grad(bool vjp, const void *params, const float *feats, const float *target, int64_t M,
                float *grads, float *work, hipStream_t st) {
    if (vjp)
        mlp_train_kernel<true><<<kTrainBlocks, kBlock, 0, st>>>(
            (const __bf16 *)params, (const float2 *)feats, target, M, 1.0f / (float)M, work);
    else
        mlp_train_kernel<false><<<kTrainBlocks, kBlock, 0, st>>>(
            (const __bf16 *)params, (const float2 *)feats, target, M, 1.0f / (float)M, work);
    const int rows = kTrainBlocks * kWaves, per = rows / kGradGroups;
    float *mid = work + (int64_t)rows * kNParams;
    grad_reduce_kernel<<<dim3((kNParams + 255) / 256, kGradGroups), 256, 0, st>>>(work, rows, per,
                                                                                  mid);
    grad_reduce_kernel<<<dim3((kNParams + 255) / 256, 1), 256, 0, st>>>(mid, kGradGroups,
                                                                        kGradGroups, grads);
    SR_HIP_CHECK(hipGetLastError());
    return SR_OK;
}

}  // namespace
}  // namespace sr

using namespace sr;

extern "C" int sr_mlp_forward(const void *params, const float *feats, float *out, int64_t M,
                              void *stream) {
    if (!params || M < 0 || (M > 0 && (!feats || !out))) return SR_E_INVAL;
    if (M == 0) return SR_OK;
    int64_t tiles = (M + 15) / 16;
    int64_t blocks = (tiles + kWaves - 1) / kWaves;
    if (blocks > 4096) blocks = 4096;
    mlp_forward_kernel<<<(unsigned)blocks, kBlock, 0, (hipStream_t)stream>>>(
        (const __bf16 *)params, (const float2 *)feats, out, M);
    SR_HIP_CHECK(hipGetLastError());
    return SR_OK;
}

extern "C" int64_t sr_mlp_grad_work(void) {
    return ((int64_t)kTrainBlocks * kWaves + kGradGroups) * kNParams;
}

extern "C" int sr_mlp_mse_grad(const void *params, const float *feats, const float *target,
                               int64_t M, float *grads, float *work, void *stream) {
    if (!params || !grads || !work || M <= 0 || !feats || !target) return SR_E_INVAL;
    return launch_grad(false, params, feats, target, M, grads, work, (hipStream_t)stream);
}

extern "C" int sr_mlp_backward(const void *params, const float *feats, const float *dout,
                               float *grads, int64_t M, float *work, void *stream) {
    if (!params || !grads || !work || M <= 0 || !feats || !dout) return SR_E_INVAL;
    return launch_grad(true, params, feats, dout, M, grads, work, (hipStream_t)stream);
}

extern "C" int64_t sr_mlp_train_work(int64_t batch) {
    if (batch <= 0) return -1;
    return 3 * batch + kNParams + sr_mlp_grad_work();
}

extern "C" int sr_mlp_train(float *master, void *params, float *m, float *v, int64_t t0,
                            const sr_table *tab, uint64_t seed, int64_t steps, int64_t batch,
                            float lr, float lr_final, int32_t kin_cut, double log10chi_lo,
                            double log10chi_hi, float *work, void *stream) {
    if (!master || !params || !m || !v || !tab || !work || t0 < 0 || steps < 0 || batch <= 0 ||
        batch > ((int64_t)1 << 26) || !(lr > 0.0f) || !(lr_final > 0.0f) ||
        !(log10chi_hi > log10chi_lo))
        return SR_E_INVAL;
    float *feats = work, *target = work + 2 * batch, *grads = work + 3 * batch;
    float *gwork = grads + kNParams;
    for (int64_t s = 0; s < steps; ++s) {
        int rc = sr_mlp_make_batch(tab, seed, (uint64_t)(t0 + s), kin_cut, log10chi_lo,
                                   log10chi_hi, feats, target, batch, stream);
        if (rc == SR_OK) rc = sr_mlp_mse_grad(params, feats, target, batch, grads, gwork, stream);
        const double frac = steps > 1 ? (double)s / (double)(steps - 1) : 0.0;
        const float cur = (float)(lr_final + 0.5 * (lr - lr_final) *
                                                 (1.0 + cos(3.14159265358979323846 * frac)));
        if (rc == SR_OK) rc = sr_mlp_adam(master, params, grads, m, v, t0 + s + 1, cur, 0.9f,
                                          0.999f, 1e-8f, stream);
        if (rc != SR_OK) return rc;
    }
    return SR_OK;
}

extern "C" int64_t sr_mlp_judge_work(int32_t n_u, int32_t chi_per_bin, int32_t n_xbins) {
    if (n_u < 1 || chi_per_bin < 1 || n_xbins < 1 || n_xbins > 4096) return -1;
    const int64_t total = (int64_t)kMlpFallbackBins * chi_per_bin * n_u;
    // floats: x_tab, network output, two features; then the FP64 histograms
    const int64_t floats = 4 * total + 4;   // keep the histograms 8-byte aligned
    return floats + 2 * (int64_t)kMlpFallbackBins * 2 * n_xbins;
}

extern "C" int sr_mlp_judge(const void *params, const sr_table *tab, int32_t kin_cut, int32_t n_u,
                            int32_t chi_per_bin, double x_lo, double x_hi, int32_t n_xbins,
                            double tol, double *err, uint8_t *fallback, float *work,
                            void *stream) {
    const int64_t need = sr_mlp_judge_work(n_u, chi_per_bin, n_xbins);
    if (!params || !tab || !err || !fallback || !work || need < 0 || !(x_lo > 0.0) ||
        !(x_hi > x_lo) || !(tol >= 0.0))
        return SR_E_INVAL;
    const int64_t total = (int64_t)kMlpFallbackBins * chi_per_bin * n_u;
    if (total > ((int64_t)1 << 30)) return SR_E_UNSUPPORTED;
    hipStream_t st = (hipStream_t)stream;
    float *x_tab = work, *y_net = work + total;
    float *feats = work + 2 * total;
    // the histograms start at the first 8-byte boundary after the floats (the
    // workspace holds four spare floats for it)
    double *hist = (double *)(((uintptr_t)(work + 4 * total) + 7) & ~(uintptr_t)7);
    const int64_t nh = (int64_t)kMlpFallbackBins * 2 * n_xbins;
    TableDev td{tab->ftab, tab->pa, tab->t1, tab->r, tab->gtab, tab->qtab};
    JudgeGrid G{n_u, chi_per_bin, (kMlpChiHi - kMlpChiLo) / (float)kMlpFallbackBins};
    judge_inputs_kernel<<<(unsigned)((total + 255) / 256), 256, 0, st>>>(td, G, kin_cut, total,
                                                                          x_tab, (float2 *)feats);
    SR_HIP_CHECK(hipGetLastError());
    const int rc = sr_mlp_forward(params, feats, y_net, total, stream);
    if (rc != SR_OK) return rc;
    zero_doubles_kernel<<<(unsigned)((nh + 255) / 256), 256, 0, st>>>(hist, nh);
    const double l_lo = log(x_lo), inv_w = (double)n_xbins / (log(x_hi) - log(x_lo));
    const int64_t per_bin = (int64_t)chi_per_bin * n_u;
    const unsigned parts = (unsigned)std::min<int64_t>((per_bin + 255) / 256, 64);
    judge_hist_kernel<<<dim3(parts, kMlpFallbackBins), 256, sizeof(double) * 2 * n_xbins, st>>>(
        G, x_tab, y_net, l_lo, inv_w, n_xbins, hist);
    judge_err_kernel<<<kMlpFallbackBins, 64, 0, st>>>(hist, n_xbins, tol, err, fallback);
    SR_HIP_CHECK(hipGetLastError());
    return SR_OK;
}

extern "C" int sr_mlp_adam(float *master, void *params, const float *grads, float *m, float *v,
                           int64_t t, float lr, float beta1, float beta2, float eps, void *stream) {
    if (!master || !params || !grads || !m || !v || t < 1) return SR_E_INVAL;
    const float c1 = (float)(1.0 / (1.0 - pow((double)beta1, (double)t)));
    const float c2 = (float)(1.0 / (1.0 - pow((double)beta2, (double)t)));
    adam_kernel<<<(kNParams + 255) / 256, 256, 0, (hipStream_t)stream>>>(
        master, (__bf16 *)params, grads, m, v, lr, beta1, beta2, eps, c1, c2);
    SR_HIP_CHECK(hipGetLastError());
    return SR_OK;
}

extern "C" int sr_mlp_cast(const float *master, void *params, void *stream) {
    if (!master || !params) return SR_E_INVAL;
    cast_kernel<<<(kNParams + 255) / 256, 256, 0, (hipStream_t)stream>>>(master, (__bf16 *)params);
    SR_HIP_CHECK(hipGetLastError());
    return SR_OK;
}

extern "C" int sr_mlp_make_batch(const sr_table *tab, uint64_t seed, uint64_t batch,
                                 int32_t kin_cut, double log10chi_lo, double log10chi_hi,
                                 float *feats, float *target, int64_t M, void *stream) {
    if (!tab || M < 0 || (M > 0 && (!feats || !target)) || !(log10chi_hi > log10chi_lo))
        return SR_E_INVAL;
    if (M == 0) return SR_OK;
    TableDev td{tab->ftab, tab->pa, tab->t1, tab->r, tab->gtab, tab->qtab};
    make_batch_kernel<<<(unsigned)((M + 255) / 256), 256, 0, (hipStream_t)stream>>>(
        td, (uint32_t)seed, (uint32_t)(seed >> 32), (uint32_t)batch, kin_cut, (float)log10chi_lo,
        (float)log10chi_hi, (float2 *)feats, target, M);
    SR_HIP_CHECK(hipGetLastError());
    return SR_OK;
}

extern "C" int sr_eval_direct(const sr_table *tab, const uint32_t *a, const float *chi,
                              int32_t kin_cut, float *out_x, int64_t n, void *stream) {
    if (!tab || n < 0 || (n > 0 && (!a || !chi || !out_x))) return SR_E_INVAL;
    if (n == 0) return SR_OK;
    TableDev td{tab->ftab, tab->pa, tab->t1, tab->r, tab->gtab, tab->qtab};
    eval_direct_kernel<<<(unsigned)((n + 255) / 256), 256, 0, (hipStream_t)stream>>>(
        td, a, chi, kin_cut, out_x, n);
    SR_HIP_CHECK(hipGetLastError());
    return SR_OK;
}
