// sr_common.hpp -- device helpers shared by the libsr kernels (gfx950, wave64).
//
// Normalised units, c = m = e = 1, electron charge q = -1.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "sr.h"

#define SR_HIP_CHECK(expr)                                   \
    do {                                                     \
        hipError_t _e = (expr);                              \
        if (_e != hipSuccess) return SR_E_HIP;               \
    } while (0)

namespace sr {

constexpr int kBlock = 256;     // threads per block, one particle each
constexpr int kWaves = kBlock / 64;
constexpr int kChunk = SR_CHUNK; // particles per chunk: one wave
constexpr int kMaxK = 16;       // largest supported number of trials per step

// Square root and reciprocal: the hardware instructions (1 ulp) in binary32,
// correctly rounded operations in FP64.
template <typename R> __device__ __forceinline__ R sqrt_r(R v);
template <> __device__ __forceinline__ float sqrt_r<float>(float v) { return __builtin_amdgcn_sqrtf(v); }
template <> __device__ __forceinline__ double sqrt_r<double>(double v) { return sqrt(v); }
template <typename R> __device__ __forceinline__ R fma_r(R a, R b, R c);
template <> __device__ __forceinline__ float fma_r<float>(float a, float b, float c) { return fmaf(a, b, c); }
template <> __device__ __forceinline__ double fma_r<double>(double a, double b, double c) { return fma(a, b, c); }
template <typename R> __device__ __forceinline__ R rcp_r(R v);
template <> __device__ __forceinline__ float rcp_r<float>(float v) { return __builtin_amdgcn_rcpf(v); }
template <> __device__ __forceinline__ double rcp_r<double>(double v) { return 1.0 / v; }

// Element access through a 32-bit byte offset from a base pointer, so the
// address is formed as (scalar base + vector offset) with no 64-bit arithmetic.
// Callers keep every array below 4 GiB.
// The accesses name the global address space, so they compile to global (not
// flat) memory instructions: flat ones also count against the LDS / scalar wait
// counter, which would make every LDS or scalar wait also wait for them.
#define SR_GLOBAL __attribute__((address_space(1)))
template <typename T>
__device__ __forceinline__ T ld(const T *base, uint32_t i) {
    return *(const SR_GLOBAL T *)((const SR_GLOBAL char *)base + i * (uint32_t)sizeof(T));
}
template <typename T>
__device__ __forceinline__ void st(T *base, uint32_t i, T v) {
    *(SR_GLOBAL T *)((SR_GLOBAL char *)base + i * (uint32_t)sizeof(T)) = v;
}

// ---------------------------------------------------------------------------
// Synchrotron-function table (built in FP64 by the table kernels, read here).
// Two families of cubic pieces in t = log2 x with 32 pieces per unit of t:
//   lower (x below the proposal branch point):  L(t) = log2( F(x) / x^{1/3} )
//   upper (x above it):                         L(t) = log2( F(x) e^{x} / x^{1/3} )
// Both stay O(1) over their ranges, so a binary32 cubic holds them to ~1e-7.
// Piece j covers t in [j/32, (j+1)/32); coefficients are for s in [0,1).
// ---------------------------------------------------------------------------
constexpr int kFPerUnit = 32;
constexpr int kFLoJ0 = -592;    // t from -18.5 (x = 2^-18.5) ...
constexpr int kFLoN = 592;      // ... to 0
constexpr int kFUpJ0 = -32;     // t from -1 ...
constexpr int kFUpN = 176;      // ... to 4.5 (x = 22.6)
constexpr int kFTotal = kFLoN + kFUpN;

// Direct samplers.  With the kinematic cut the photon-number CDF is
// N(x)/N(xmax(chi)), N(x) = int_0^x F(t)/t dt, xmax = 2/(3 chi); hence
// x = T1(U) with U = u r(chi), r = N(xmax)/N(inf), T1 the uncut inverse CDF.
//   T1: cubic pieces of y = log2 x in w = logit(U) on [-kT1W, kT1W].
//   r : r(chi) and 1 - r(chi) on log10 chi nodes, linear between nodes.
constexpr int kT1N = 6144;              // pieces of T1 (128 per unit of logit)
constexpr double kT1W = 24.0;           // logit range: U down to 3.8e-11
constexpr int kRPerDecade = 512;
constexpr double kRLogChiLo = -6.0;     // below: r = 1 to binary32 precision
constexpr double kRLogChiHi = 4.0;      // above: r ~ chi^{-1/3} (small-x form of N)
constexpr int kRN = (int)((kRLogChiHi - kRLogChiLo) * kRPerDecade) + 1;

// Trial-density table of the proposal, for the emission kernel: the density
// q = F(x)/(x S(x)) of one trial as a function of the uniform R' itself, so a
// trial costs one logarithm, one cubic and one exponential.  Cubic pieces of
// log2 q with 32 pieces per unit of the argument:
//   lower family (R' <= P(a)):  argument u = log2 R',       x = 2^{3u/4}
//   upper family:               argument v = -log2(1 - R'), x = v ln2 - ln(9/7)
constexpr int kGPerUnit = 32;
constexpr int kGLoJ0 = -768;    // u from -24 (R' = 2^-24) ...
constexpr int kGLoN = 768;      // ... to 0
constexpr int kGUpJ0 = 32;      // v from 1 ...
constexpr int kGUpN = 736;      // ... to 24 (1 - R' = 2^-24)
constexpr int kGTotal = kGLoN + kGUpN;

// Quantum-corrected kernel table (the quantum synchrotron spectrum for chi
// approaching 1, where section "Limitations" says the classical expression
// fails).  With delta = 1.5 chi x and xi = x/(1 - delta) the per-unit-x kernel
// is Q = (1 - delta + 1/(1 - delta)) K_{2/3}(xi) - int_xi^inf K_{1/3}.  Piece j
// of t = log2 xi on [-19, 7) holds, as Hermite cubics in the local coordinate,
//   qtab[2j]   : yA = log2 K_{2/3}(xi) + (2/3) t + xi log2 e
//   qtab[2j+1] : yB = log2 int_xi^inf K_{1/3} + xi log2 e
// (both slowly varying: the xi^{-2/3} and e^{-xi} behaviour is taken out).
// xi >= 2^-18 always (x >= the proposal's smallest x); above xi = 128 the
// kernel is below e^-128 and the trial is taken as dN = 0.
constexpr int kQPerUnit = 16;
constexpr int kQJ0 = -19 * kQPerUnit;
constexpr int kQN = 26 * kQPerUnit;
constexpr float kQXiMax = 128.0f;

struct TableDev {
    const float4 *ftab;     // [kFTotal]
    float pa;               // binary32 branch point P(a)
    const float4 *t1;       // [kT1N]
    const float2 *r;        // [kRN] (r, 1 - r)
    const float4 *gtab;     // [kGTotal]
    const float4 *qtab;     // [2 * kQN]
};

// ---------------------------------------------------------------------------
// Philox4x32-10 (Salmon, Moraes, Dror & Shaw, SC'11).
// ---------------------------------------------------------------------------
// A wave-uniform value the optimiser cannot see through: a loop bound tested
// each trial as a scalar compare, rather than kept as a precomputed lane mask
// per trial in scalar registers.
__device__ __forceinline__ int uniform_opaque(int v) {
    asm volatile("" : "+s"(v));
    return v;
}

// a ^ b ^ c in one VALU instruction (gfx950 three-input bit operation; the
// truth table 0x96 is the XOR of its three inputs)
__device__ __forceinline__ uint32_t xor3(uint32_t a, uint32_t b, uint32_t c) {
    return __builtin_amdgcn_bitop3_b32(a, b, c, 0x96);
}

// The key (k0, k1) must be wave-uniform.  The empty asm hides it from the
// optimiser, so each call steps the key schedule with scalar adds instead of
// keeping all twenty round keys live in scalar registers across the kernel.
__device__ __forceinline__ uint4 philox4x32_10(uint4 c, uint32_t k0, uint32_t k1) {
    asm volatile("" : "+s"(k0), "+s"(k1));
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        if (r) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        const uint64_t m0 = (uint64_t)0xD2511F53u * c.x;
        const uint64_t m1 = (uint64_t)0xCD9E8D57u * c.z;
        if (r == 0) {
            c = make_uint4((uint32_t)(m1 >> 32) ^ c.y ^ k0, (uint32_t)m1,
                           (uint32_t)(m0 >> 32) ^ c.w ^ k1, (uint32_t)m0);
        } else {
            c = make_uint4(xor3((uint32_t)(m1 >> 32), c.y, k0), (uint32_t)m1,
                           xor3((uint32_t)(m0 >> 32), c.w, k1), (uint32_t)m0);
        }
    }
    return c;
}

// ---------------------------------------------------------------------------
// F-table lookup.
// ---------------------------------------------------------------------------
__device__ __forceinline__ float ftab_eval(const float4 *__restrict__ tab, float t, int j0, int n,
                                           int base) {
    const float u = t * (float)kFPerUnit;   // exact scaling
    const float fj = floorf(u);
    int j = (int)fj - j0;
    j = min(max(j, 0), n - 1);
    const float s = u - (float)(j + j0);    // exact for in-range t
    const float4 c = tab[base + j];
    return fmaf(fmaf(fmaf(c.w, s, c.z), s, c.y), s, c.x);
}

// One trial with the proposal S(x), through the trial-density table: returns
// q = F(x)/(x S(x)) at the R' of word a (a 23-bit midpoint, never 0 or 1), and
// lg = log2 R' on the lower branch or log2(1 - R') on the upper one, from which
// trial_x gives x.  dN = rate q (the dN of the recipe at the end of section
// "Monte Carlo method", per unit x).
__device__ __forceinline__ float trial_q(uint32_t a, const float4 *__restrict__ gtab, float pa,
                                         float &lg, bool &lower) {
    const float rp = (float)((a >> 9) * 2u + 1u) * 0x1p-24f;
    lower = rp <= pa;
    lg = __builtin_amdgcn_logf(lower ? rp : 1.0f - rp);   // 1 - rp is exact
    const float u = (lower ? lg : -lg) * (float)kGPerUnit;
    const int j0 = lower ? kGLoJ0 : kGUpJ0;
    int j = (int)floorf(u) - j0;
    j = min(max(j, 0), (lower ? kGLoN : kGUpN) - 1);
    const float s = u - (float)(j + j0);
    const float4 c = gtab[(lower ? 0 : kGLoN) + j];
    return __builtin_amdgcn_exp2f(fmaf(fmaf(fmaf(c.w, s, c.z), s, c.y), s, c.x));
}

// The pieces of the trial-density table that almost every trial reads, which
// the proposal sampler's kernels with four or more trials keep in LDS: log2 R'
// in [-8, 0) on the lower branch (256 pieces) and -log2(1 - R') in [1, 10) on
// the upper one (288 pieces), 8.7 KB.  With R' uniform, 99.4% and 99.8% of a
// branch's trials fall there.  Element e of the LDS copy holds
// gtab[ghot_source(e)].
constexpr int kGHotLo = 256;
constexpr int kGHotUp = 288;
constexpr int kGHot = kGHotLo + kGHotUp;
__device__ __forceinline__ int ghot_source(int e) {
    return e < kGHotLo ? kGLoN - kGHotLo + e : kGLoN + (e - kGHotLo);
}

// A 16-byte global load that the optimiser cannot merge with another load into
// one generic (flat) access: written out, and waited for in the same statement.
__device__ __forceinline__ float4 ld_global_wait(const float4 *p) {
    float4 v;
    asm volatile("global_load_dwordx4 %0, %1, off\n\ts_waitcnt vmcnt(0)" : "=v"(v) : "v"(p)
                 : "memory");
    return v;
}

// trial_q with the hot pieces read from their LDS copy ghot: the same values,
// so the same result.  Every lane reads the LDS copy (the cold lanes at a
// clamped index) and only the rare cold lanes then read the table in global
// memory, as a separate load.
__device__ __forceinline__ float trial_q_hot(uint32_t a, const float4 *__restrict__ gtab,
                                             const float4 *ghot, float pa, float &lg,
                                             bool &lower) {
    const float rp = (float)((a >> 9) * 2u + 1u) * 0x1p-24f;
    lower = rp <= pa;
    lg = __builtin_amdgcn_logf(lower ? rp : 1.0f - rp);   // 1 - rp is exact
    const float u = (lower ? lg : -lg) * (float)kGPerUnit;
    const int j0 = lower ? kGLoJ0 : kGUpJ0;
    int j = (int)floorf(u) - j0;
    j = min(max(j, 0), (lower ? kGLoN : kGUpN) - 1);
    const float s = u - (float)(j + j0);
    // LDS index: the lower pieces at j - (kGLoN - kGHotLo), always below
    // kGHotLo, and the upper ones at kGHotLo + j, never below it; so a piece
    // is hot exactly when its index lies in [0, kGHot)
    const int idx = j + (lower ? kGHotLo - kGLoN : kGHotLo);
    const bool hot = (uint32_t)idx < (uint32_t)kGHot;
    float4 c = ghot[hot ? idx : 0];
    if (!hot) c = ld_global_wait(gtab + (lower ? 0 : kGLoN) + j);
    return __builtin_amdgcn_exp2f(fmaf(fmaf(fmaf(c.w, s, c.z), s, c.y), s, c.x));
}

// x of a trial (word a, trial_q's lg): R'^{3/4} as sqrt(R') sqrt(sqrt(R'))
// (a few ulp, where 2^{3 lg/4} would lose ~1e-6 to the rounding of lg), or
// -ln((9/7)(1 - R')).
__device__ __forceinline__ float trial_x(uint32_t a, float lg, bool lower) {
    if (lower) {
        const float rp = (float)((a >> 9) * 2u + 1u) * 0x1p-24f;
        const float s = __builtin_amdgcn_sqrtf(rp);
        return s * __builtin_amdgcn_sqrtf(s);
    }
    return fmaf(-0.69314718055994531f, lg, -0.25131442828090605f);
}

// Quantum trial: dN / rate = Q(x, chi) / S(x) at the proposal's x(R') (the
// classical recipe with the quantum kernel in place of F(x)/x), and x itself.
// Zero at and above the kinematic edge delta = 1.5 chi x >= 1.
//
// With HOT, the pieces of log2 xi >= -6 (kQHot0 on: 208 pieces, 6.7 KB, which
// all but ~0.4% of the trials read) come from their LDS copy qhot, element e
// holding qtab[2 kQHot0 + e]; the rare colder lanes read the global table with
// separate loads.  The same values either way, so the same result.
constexpr int kQHot0 = (-6 * kQPerUnit) - kQJ0;
constexpr int kQHot = 2 * (kQN - kQHot0);
template <bool HOT>
__device__ __forceinline__ float quantum_q_t(uint32_t a, const float4 *__restrict__ qtab,
                                             const float4 *qhot, float pa, float chi, float &x) {
    const float rp = (float)((a >> 9) * 2u + 1u) * 0x1p-24f;
    const bool lower = rp <= pa;
    const float lg = __builtin_amdgcn_logf(lower ? rp : 1.0f - rp);
    x = trial_x(a, lg, lower);
    // log2(1/S): lower S = (4/3) R'^{1/4}, upper S = 1 - R'
    const float l2_inv_s = lower ? -fmaf(0.25f, lg, 0.41503749927884381f) : -lg;
    const float delta = 1.5f * chi * x;
    if (!(delta < 1.0f)) return 0.0f;
    const float om = 1.0f - delta;
    const float xi = x / om;
    if (!(xi < kQXiMax)) return 0.0f;
    const float t = __builtin_amdgcn_logf(xi);
    const float u = t * (float)kQPerUnit;
    int j = (int)floorf(u) - kQJ0;
    j = min(max(j, 0), kQN - 1);
    const float s = u - (float)(j + kQJ0);
    float4 ca, cb;
    if constexpr (HOT) {
        const int h = 2 * max(j - kQHot0, 0);
        ca = qhot[h];
        cb = qhot[h + 1];
        if (j < kQHot0) {
            ca = ld_global_wait(qtab + 2 * j);
            cb = ld_global_wait(qtab + 2 * j + 1);
        }
    } else {
        ca = qtab[2 * j];
        cb = qtab[2 * j + 1];
    }
    const float ya = fmaf(fmaf(fmaf(ca.w, s, ca.z), s, ca.y), s, ca.x);
    const float yb = fmaf(fmaf(fmaf(cb.w, s, cb.z), s, cb.y), s, cb.x);
    const float c = om + 1.0f / om;
    const float q = c * __builtin_amdgcn_exp2f(fmaf(-0.66666666666666667f, t, ya)) -
                    __builtin_amdgcn_exp2f(yb);
    return q * __builtin_amdgcn_exp2f(fmaf(-1.4426950408889634f, xi, l2_inv_s));
}
__device__ __forceinline__ float quantum_q(uint32_t a, const float4 *__restrict__ qtab, float pa,
                                           float chi, float &x) {
    return quantum_q_t<false>(a, qtab, nullptr, pa, chi, x);
}

// Kinematic cut x > xc = 2/(3 chi) expressed on lg: on the lower branch
// lg > (4/3) log2 xc, on the upper one lg < -(xc + ln(9/7))/ln2.  Without the
// cut (or chi = 0) nothing is cut.
struct TrialCut {
    float lo, hi;
};
__device__ __forceinline__ TrialCut trial_cut(bool on, float chi) {
    TrialCut c{__builtin_inff(), -__builtin_inff()};
    if (on && chi > 0.0f) {
        const float xc = __builtin_amdgcn_rcpf(1.5f * chi);
        c.lo = -1.3333333333333333f * __builtin_amdgcn_logf(1.5f * chi);
        c.hi = -(xc + 0.25131442828090605f) * 1.4426950408889634f;
    }
    return c;
}
__device__ __forceinline__ bool trial_is_cut(const TrialCut &c, float lg, bool lower) {
    return lower ? lg > c.lo : lg < c.hi;
}
// Grid floor x < xf = e_grid / eps_unit on lg: on the lower branch lg <
// (4/3) log2 xf, on the upper one lg > -(xf + ln(9/7))/ln2.  The bounds come
// back in a TrialCut: below lo (lower) or above hi (upper) is under the floor.
__device__ __forceinline__ TrialCut trial_floor(float e_grid, float eps_unit) {
    TrialCut c{-__builtin_inff(), __builtin_inff()};
    if (eps_unit > 0.0f) {
        const float xf = e_grid / eps_unit;
        c.lo = 1.3333333333333333f * __builtin_amdgcn_logf(xf);
        c.hi = -(xf + 0.25131442828090605f) * 1.4426950408889634f;
    }
    return c;
}
__device__ __forceinline__ bool trial_is_floored(const TrialCut &c, float lg, bool lower) {
    return lower ? lg < c.lo : lg > c.hi;
}

// r(chi) and 1 - r(chi), linear in log10 chi; r ~ chi^{-1/3} above the table.
__device__ __forceinline__ float2 r_lookup(const float2 *__restrict__ rt, float chi) {
    if (!(chi > 0.0f)) return make_float2(1.0f, 0.0f);
    const float u = (__log2f(chi) * 0.30102999566398120f - (float)kRLogChiLo) * (float)kRPerDecade;
    if (u <= 0.0f) return rt[0];
    if (u >= (float)(kRN - 1)) {
        const float r = rt[kRN - 1].x * exp2f((float)(kRN - 1 - u) * (1.0f / 3.0f) *
                                              (3.3219280948873623f / kRPerDecade));
        return make_float2(r, 1.0f - r);
    }
    const int j = (int)u;
    const float s = u - (float)j;
    const float2 a = rt[j], b = rt[j + 1];
    return make_float2(fmaf(s, b.x - a.x, a.x), fmaf(s, b.y - a.y, a.y));
}

// x = T1(U) from ln U and ln(1-U) (the uncut inverse number-CDF).
__device__ __forceinline__ float t1_log2x(const float4 *__restrict__ t1, float lnU, float ln1mU) {
    const float w = lnU - ln1mU;
    const float u = (w + (float)kT1W) * (float)(kT1N / (2.0 * kT1W));
    int j = (int)floorf(u);
    j = min(max(j, 0), kT1N - 1);
    const float s = u - (float)j;
    const float4 c = t1[j];
    return fmaf(fmaf(fmaf(c.w, s, c.z), s, c.y), s, c.x);
}

// ln U and ln(1-U) for U = u r with u a 23-bit midpoint from word a and
// (r, 1-r) from r_lookup: 1 - U = (1-u) + u (1-r) keeps the upper tail exact.
__device__ __forceinline__ void direct_u(uint32_t a, float2 r, float &lnU, float &ln1mU) {
    const float u = (float)((a >> 9) * 2u + 1u) * 0x1p-24f;
    const float om = 1.0f - u;  // exact
    lnU = 0.69314718055994531f * (__log2f(u) + __log2f(r.x));
    ln1mU = 0.69314718055994531f * __log2f(fmaf(u, r.y, om));
}

// ---------------------------------------------------------------------------
// Grid description passed to the kernels.
// ---------------------------------------------------------------------------
struct GridK {
    int dim;
    int n[3];
    float inv_hi[3], inv_lo[3];   // 1/dx split into a binary32 pair
    double inv_d[3];              // 1/dx in FP64 (FP64 path)
    float L[3];                   // box lengths (binary32)
    double Ld[3];                 // box lengths (FP64)
    float e0[3], b0[3];           // uniform fields (dim 0)
    double e0d[3], b0d[3];
};

// Cell index and fraction of a coordinate for nodes at offset 0 and 1/2.
template <typename R>
struct Axis {
    int i0, i1;    // base nodes (wrapped) for offset 0 and 1/2
    int i0p, i1p;  // next nodes (wrapped)
    R f0, f1;      // fractions
};

// One periodic wrap, then a clamp so that even a corrupt position (NaN, far
// outside the box) can never index outside the grid.
__device__ __forceinline__ int wrap_i(int i, int n) {
    i = i < 0 ? i + n : (i >= n ? i - n : i);
    return min(max(i, 0), n - 1);
}

// binary32: u = x/dx with the product split so the fraction keeps ~2^-24 absolute accuracy
__device__ __forceinline__ void axis_setup(float x, float inv_hi, float inv_lo, int n,
                                           Axis<float> &ax) {
    const float u = x * inv_hi;
    float fi = floorf(u);
    float f = fmaf(x, inv_hi, -fi) + x * inv_lo;
    if (f < 0.0f) { f += 1.0f; fi -= 1.0f; }
    if (f >= 1.0f) { f -= 1.0f; fi += 1.0f; }
    int i0 = (int)fi;
    int i1;
    float f1;
    if (f >= 0.5f) { i1 = i0; f1 = f - 0.5f; } else { i1 = i0 - 1; f1 = f + 0.5f; }
    ax.i0 = wrap_i(i0, n);
    ax.i0p = wrap_i(ax.i0 + 1, n);
    ax.i1 = wrap_i(i1, n);
    ax.i1p = wrap_i(ax.i1 + 1, n);
    ax.f0 = f;
    ax.f1 = f1;
}

__device__ __forceinline__ void axis_setup(double x, double inv, int n, Axis<double> &ax) {
    const double u = x * inv;
    double fi = floor(u);
    double f = u - fi;
    int i0 = (int)fi;
    int i1;
    double f1;
    if (f >= 0.5) { i1 = i0; f1 = f - 0.5; } else { i1 = i0 - 1; f1 = f + 0.5; }
    ax.i0 = wrap_i(i0, n);
    ax.i0p = wrap_i(ax.i0 + 1, n);
    ax.i1 = wrap_i(i1, n);
    ax.i1p = wrap_i(ax.i1 + 1, n);
    ax.f0 = f;
    ax.f1 = f1;
}

// Two consecutive grid values of a row from one 8-byte load (4-byte aligned).
typedef float f32x2_a4 __attribute__((ext_vector_type(2), aligned(4)));
__device__ __forceinline__ float2 ld2(const float *base, uint32_t i) {
    const f32x2_a4 v = *(const SR_GLOBAL f32x2_a4 *)((const SR_GLOBAL char *)base + i * 4u);
    return make_float2(v.x, v.y);
}

// The two x-neighbours (ix, ix+1 periodic) of every row of a component, read
// as pairs: rows need nx >= 2; the pair starts at min(ix, nx-2), and the lanes
// at ix = nx-1 (whose right neighbour wraps to 0) fix theirs up with one more
// load, issued only when some lane of the wave wraps.
struct XPair {
    uint32_t start;   // first element of the loaded pair
    bool wrap;        // ix == nx - 1
    bool any_wrap;    // some lane of the wave wraps (wave-uniform)
};
__device__ __forceinline__ XPair x_pair(uint32_t ix, int nx) {
    XPair p;
    p.wrap = ix == (uint32_t)(nx - 1);
    p.start = p.wrap ? (uint32_t)(nx - 2) : ix;
    p.any_wrap = __ballot(p.wrap) != 0;
    return p;
}
template <typename R>
__device__ __forceinline__ R row_lerp(const float *__restrict__ a, uint32_t row, const XPair &p,
                                      R gx, R fx) {
    const float2 v = ld2(a, row + p.start);
    float lo = v.x, hi = v.y;
    if (p.any_wrap && p.wrap) {
        lo = v.y;
        hi = ld(a, row);
    }
    return fma_r<R>(gx, (R)lo, fx * (R)hi);
}

// The trilinear combination of four interpolated rows, with its roundings
// fixed (explicit fused multiply-adds) so that the direct and the LDS-box
// gathers give the same bits.
template <typename R>
__device__ __forceinline__ R trilerp(R gy, R fy, R gz, R fz, R c00, R c01, R c10, R c11) {
    return fma_r<R>(gz, fma_r<R>(gy, c00, fy * c01), fz * fma_r<R>(gy, c10, fy * c11));
}

// Bilinear (2D) / trilinear (3D) interpolation of one component.  sx, sy, sz
// select offset 0 (false) or 1/2 (true) on each axis; P0 / P1 are the x pairs
// of the two offsets.
template <typename R, int DIM>
__device__ __forceinline__ R cic(const float *__restrict__ a, const Axis<R> &X, const Axis<R> &Y,
                                 const Axis<R> &Z, const XPair &P0, const XPair &P1, bool sx,
                                 bool sy, bool sz, int nx, int ny) {
    const XPair &P = sx ? P1 : P0;
    const R fx = sx ? X.f1 : X.f0;
    const uint32_t iy0 = sy ? Y.i1 : Y.i0, iy1 = sy ? Y.i1p : Y.i0p;
    const R fy = sy ? Y.f1 : Y.f0;
    const R gx = (R)1 - fx, gy = (R)1 - fy;
    if (DIM == 2) {
        const uint32_t r0 = __umul24(iy0, (uint32_t)nx), r1 = __umul24(iy1, (uint32_t)nx);
        return fma_r<R>(gy, row_lerp<R>(a, r0, P, gx, fx), fy * row_lerp<R>(a, r1, P, gx, fx));
    } else {
        const uint32_t iz0 = sz ? Z.i1 : Z.i0, iz1 = sz ? Z.i1p : Z.i0p;
        const R fz = sz ? Z.f1 : Z.f0;
        const R gz = (R)1 - fz;
        // rows (ny nz) and nx below 2^24, cells below 2^30: the 24-bit
        // products are exact
        const uint32_t z0 = __umul24(iz0, (uint32_t)ny), z1 = __umul24(iz1, (uint32_t)ny);
        const uint32_t p00 = __umul24(z0 + iy0, (uint32_t)nx), p01 = __umul24(z0 + iy1, (uint32_t)nx);
        const uint32_t p10 = __umul24(z1 + iy0, (uint32_t)nx), p11 = __umul24(z1 + iy1, (uint32_t)nx);
        const R c00 = row_lerp<R>(a, p00, P, gx, fx), c01 = row_lerp<R>(a, p01, P, gx, fx);
        const R c10 = row_lerp<R>(a, p10, P, gx, fx), c11 = row_lerp<R>(a, p11, P, gx, fx);
        return trilerp<R>(gy, fy, gz, fz, c00, c01, c10, c11);
    }
}

// ---------------------------------------------------------------------------
// Field box in LDS (3D, the SR_GATHER_BOX gather): the grid values of every
// node a block's stencils read, for the six components, copied once per block
// with coalesced loads.  The box covers nodes lo[a] .. lo[a] + ext[a] - 1
// (periodic) on each axis and stores component c at
// box[c][(lz ext[1] + ly) ext[0] + lx].
// ---------------------------------------------------------------------------
struct FieldBox {
    int lo[3];
    int ext[3];
};
constexpr int kBoxCells = SR_FIELD_BOX_NODES;

// Local box index of node i (in [0, n)) on an axis whose box starts at lo.
__device__ __forceinline__ uint32_t box_local(int i, int lo, int n) {
    const int l = i - lo;
    return (uint32_t)(l < 0 ? l + n : l);
}

// One component from the box, with the values and the arithmetic of
// cic<R, 3>: bit-identical to the direct gather.
template <typename R>
__device__ __forceinline__ R cic_box(const float *__restrict__ b, const Axis<R> &X,
                                     const Axis<R> &Y, const Axis<R> &Z, const FieldBox &B,
                                     const int n[3], bool sx, bool sy, bool sz) {
    const uint32_t lx = box_local(sx ? X.i1 : X.i0, B.lo[0], n[0]);
    const R fx = sx ? X.f1 : X.f0;
    const uint32_t y0 = box_local(sy ? Y.i1 : Y.i0, B.lo[1], n[1]);
    const R fy = sy ? Y.f1 : Y.f0;
    const uint32_t z0 = box_local(sz ? Z.i1 : Z.i0, B.lo[2], n[2]);
    const R fz = sz ? Z.f1 : Z.f0;
    const R gx = (R)1 - fx, gy = (R)1 - fy, gz = (R)1 - fz;
    const uint32_t ex = (uint32_t)B.ext[0], ey = (uint32_t)B.ext[1];
    const uint32_t r00 = (z0 * ey + y0) * ex + lx;
    const uint32_t r01 = r00 + ex, r10 = r00 + ex * ey, r11 = r10 + ex;
    const auto lerp = [&](uint32_t r) { return fma_r<R>(gx, (R)b[r], fx * (R)b[r + 1]); };
    const R c00 = lerp(r00), c01 = lerp(r01), c10 = lerp(r10), c11 = lerp(r11);
    return trilerp<R>(gy, fy, gz, fz, c00, c01, c10, c11);
}

// a*b - c*d with one rounding error (Kahan's fused algorithm).
__device__ __forceinline__ float diff_of_products(float a, float b, float c, float d) {
    const float w = c * d;
    const float e = fmaf(-c, d, w);
    const float f = fmaf(a, b, -w);
    return f + e;
}
__device__ __forceinline__ double diff_of_products(double a, double b, double c, double d) {
    return a * b - c * d;
}

// ---------------------------------------------------------------------------
// Wave64 reductions.
// ---------------------------------------------------------------------------
}  // namespace sr
// Whole-wave reductions of the device library (DPP row shifts and broadcasts,
// fixed order); every lane of the wave must be active.
extern "C" __device__ __attribute__((const)) double __ockl_wfred_add_f64(double);
extern "C" __device__ __attribute__((const)) float __ockl_wfred_max_f32(float);
extern "C" __device__ __attribute__((const)) float __ockl_wfred_add_f32(float);
namespace sr {
__device__ __forceinline__ double wave_sum(double v) { return __ockl_wfred_add_f64(v); }
__device__ __forceinline__ float wave_max(float v) { return __ockl_wfred_max_f32(v); }
__device__ __forceinline__ float wave_sum_f(float v) { return __ockl_wfred_add_f32(v); }
__device__ __forceinline__ int wave_min_i(int v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = min(v, __shfl_xor(v, o, 64));
    return v;
}
__device__ __forceinline__ int wave_max_i(int v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = max(v, __shfl_xor(v, o, 64));
    return v;
}
__device__ __forceinline__ uint32_t lane_prefix(uint64_t mask) {
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32),
                                     __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}

// Logical chunk for a block so that chunks adjacent in memory land on the same
// XCD (blocks are dealt round-robin to the 8 XCDs).
__device__ __forceinline__ int64_t xcd_chunk(int64_t b, int64_t G) {
    const int64_t q = G / 8, r = G % 8;
    const int64_t xcd = b % 8, local = b / 8;
    return xcd < r ? xcd * (q + 1) + local : r * (q + 1) + (xcd - r) * q + local;
}

}  // namespace sr

// Host-side table object.
struct sr_table {
    float4 *ftab = nullptr;
    float4 *gtab = nullptr;
    float4 *qtab = nullptr;
    float4 *t1 = nullptr;
    float2 *r = nullptr;
    float pa = 0.0f;
    double a = 0.0;
    int device = 0;
};
