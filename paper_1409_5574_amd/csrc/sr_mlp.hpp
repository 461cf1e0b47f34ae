// sr_mlp.hpp -- device side of the MLP surrogate for the inverse number-CDF.
//
// Network: features (f0, f1) -> 64 -> SiLU -> 64 -> SiLU -> 64 -> SiLU -> 1,
// output log2 x.  f0 = (log10 chi + 1)/3, f1 = logit(u)/16.  Parameters are one flat
// bfloat16 vector: W1[64][2], b1[64], W2[64][64], b2[64], W3[64][64], b3[64],
// W4[64], b4 (8577 values).  The two 64x64 layers run on the matrix cores
// (v_mfma_f32_16x16x32_bf16: bfloat16 inputs, FP32 accumulation) over tiles of
// 16 samples per wave; the 2->64 and 64->1 layers are FP32 vector code.
#pragma once

#include "sr_common.hpp"

namespace sr {

typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8;
typedef __attribute__((__vector_size__(4 * sizeof(__bf16)))) __bf16 bf16x4;
typedef __attribute__((__vector_size__(4 * sizeof(float)))) float f32x4;

constexpr int kH = 64;
constexpr int kOffW1 = 0, kOffB1 = 128, kOffW2 = 192, kOffB2 = 4288, kOffW3 = 4352,
              kOffB3 = 8448, kOffW4 = 8512, kOffB4 = 8576, kNParams = 8577;

// Fallback map: per bin of log10 chi on [kMlpChiLo, kMlpChiHi) a flag that sends
// the samples of that bin to the table sampler instead of the network.
constexpr int kMlpFallbackBins = 24;
constexpr float kMlpChiLo = -4.0f, kMlpChiHi = 2.0f;
constexpr float kMlpLog2xFloor = -16.609640f;   // training targets clipped at x = 1e-5

struct alignas(16) MlpSmem {
    alignas(16) __bf16 W2[kH * kH];   // row j holds the weights of output j
    alignas(16) __bf16 W3[kH * kH];
    float W1[2 * kH];
    float b1[kH], b2[kH], b3[kH], W4[kH];
    float b4;
};

__device__ __forceinline__ float silu(float z) {
    return z * __builtin_amdgcn_rcpf(1.0f + __expf(-z));
}

// Wave-scope ordering of LDS writes before reads by other lanes of the wave.
__device__ __forceinline__ void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
    __builtin_amdgcn_wave_barrier();
}

__device__ __forceinline__ void mlp_load(MlpSmem &s, const __bf16 *__restrict__ p, int tid, int nt) {
    for (int i = tid; i < kH * kH / 8; i += nt) {
        ((bf16x8 *)s.W2)[i] = *(const bf16x8 *)(p + kOffW2 + 8 * i);
        ((bf16x8 *)s.W3)[i] = *(const bf16x8 *)(p + kOffW3 + 8 * i);
    }
    for (int i = tid; i < 2 * kH; i += nt) s.W1[i] = (float)p[kOffW1 + i];
    for (int i = tid; i < kH; i += nt) {
        s.b1[i] = (float)p[kOffB1 + i];
        s.b2[i] = (float)p[kOffB2 + i];
        s.b3[i] = (float)p[kOffB3 + i];
        s.W4[i] = (float)p[kOffW4 + i];
    }
    if (tid == 0) s.b4 = (float)p[kOffB4];
}

// Activations enter the matrix cores as a pair of bfloat16 values (hi + lo,
// two products), which keeps ~16 significant bits: the weights are bfloat16
// by definition, the activations need not be rounded that coarsely.
struct Split8 {
    bf16x8 hi, lo;
};
__device__ __forceinline__ void split_set(Split8 &s, int e, float v) {
    const __bf16 h = (__bf16)v;
    s.hi[e] = h;
    s.lo[e] = (__bf16)(v - (float)h);
}
__device__ __forceinline__ f32x4 mfma_split(const Split8 &a, const bf16x8 &b, f32x4 acc) {
    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a.hi, b, acc, 0, 0, 0);
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a.lo, b, acc, 0, 0, 0);
}

// Forward pass of 16 samples by one wave.  Lane l works on sample r = l & 15
// (the four lanes sharing r pass the same features); g = l >> 4.  tb is a
// per-wave LDS buffer of 2 x 16 x 64 bfloat16.  Returns log2 x of sample r.
//
// Matrix-core operand layout (16x16x32): A[i][k] sits in lane i + 16 (k/8 mod 4)
// as element k mod 8 of K-block k/32; B[k][j] likewise in lane j + 16 (...); the
// 16x16 FP32 result D[i][j] sits in lane j + 16 (i/4), element i mod 4.
__device__ __forceinline__ float mlp_tile16(const MlpSmem &s, __bf16 *tb, float f0, float f1) {
    const int l = threadIdx.x & 63, r = l & 15, g = l >> 4;
    Split8 a[2];
#pragma unroll
    for (int kb = 0; kb < 2; ++kb)
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            const int k = 32 * kb + 8 * g + e;
            split_set(a[kb], e, silu(fmaf(s.W1[2 * k], f0, fmaf(s.W1[2 * k + 1], f1, s.b1[k]))));
        }
    // layer 2
    f32x4 acc[4];
#pragma unroll
    for (int n = 0; n < 4; ++n) {
        acc[n] = (f32x4){0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int kb = 0; kb < 2; ++kb) {
            const bf16x8 b = *(const bf16x8 *)&s.W2[(16 * n + r) * kH + 32 * kb + 8 * g];
            acc[n] = mfma_split(a[kb], b, acc[n]);
        }
    }
    // to the A layout through LDS: hi part in tb[0..1023], lo part in tb[1024..2047]
#pragma unroll
    for (int n = 0; n < 4; ++n)
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const float v = silu(acc[n][q] + s.b2[16 * n + r]);
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
    // layer 3
#pragma unroll
    for (int n = 0; n < 4; ++n) {
        acc[n] = (f32x4){0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int kb = 0; kb < 2; ++kb) {
            const bf16x8 b = *(const bf16x8 *)&s.W3[(16 * n + r) * kH + 32 * kb + 8 * g];
            acc[n] = mfma_split(a[kb], b, acc[n]);
        }
    }
    // layer 4: per row partial dot products, summed over the 16 lanes of the group
    float sq[4] = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int n = 0; n < 4; ++n) {
        const float w4 = s.W4[16 * n + r], b3 = s.b3[16 * n + r];
#pragma unroll
        for (int q = 0; q < 4; ++q) sq[q] = fmaf(w4, silu(acc[n][q] + b3), sq[q]);
    }
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
        for (int o = 8; o > 0; o >>= 1) sq[q] += __shfl_xor(sq[q], o, 64);
    // sample r's output lives in group r/4, element r mod 4
    float y = 0.f;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const float v = __shfl(sq[q], 16 * (r >> 2), 64);
        if ((r & 3) == q) y = v;
    }
    return y + s.b4;
}

__device__ __forceinline__ float mlp_feature_chi(float chi) {
    return (__log2f(chi) * 0.30102999566398120f + 1.0f) * (1.0f / 3.0f);
}

// Input encoding of the uniform u (a 23-bit midpoint of word a): logit(u)/16,
// which keeps both ends of the inverse CDF (x ~ u^3 and x ~ -ln(1-u)) smooth.
__device__ __forceinline__ float mlp_feature_u(uint32_t a) {
    const float u = (float)((a >> 9) * 2u + 1u) * 0x1p-24f;
    return (__log2f(u) - __log2f(1.0f - u)) * (0.69314718055994531f / 16.0f);
}

}  // namespace sr
