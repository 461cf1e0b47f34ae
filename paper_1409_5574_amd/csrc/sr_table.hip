// sr_table.hip -- FP64 construction of the spectrum tables on the GPU, and the
// small evaluation entry points that expose the device samplers to tests.
//
// Everything here follows the synchrotron function of section "Modelling the
// relativistic case", F(x) = x int_x^inf K_{5/3}(t) dt, written with
// K_nu(x) = int_0^inf exp(-x cosh s) cosh(nu s) ds:
//   F(x)        = x int_0^inf exp(-x cosh s) cosh(5s/3) / cosh s ds
//   int_x^inf F(t)/t dt = int_0^inf exp(-x cosh s) cosh(5s/3) / cosh^2 s ds
// Each integrand is analytic in |Im s| < pi/2, so the trapezoid rule with step
// 1/16 is accurate to far below FP64 rounding.
#include <math.h>

#include <new>

#include "sr_common.hpp"

namespace sr {
namespace {

constexpr double kH = 1.0 / 16.0;
constexpr double kNInf = 5.2359877559829887;   // int_0^inf F(x)/x dx = 5 pi / 3

__device__ double lncosh(double y) {
    y = fabs(y);
    return y + log1p(exp(-2.0 * y)) - 0.69314718055994531;
}

// F(x) and K_{5/3}(x)
__device__ void synch_FK(double x, double &F, double &K) {
    const double s_peak = asinh(5.0 / (3.0 * x));
    double sF = 0.0, sK = 0.0;
    for (int j = 0; j < 200000; ++j) {
        const double s = j * kH;
        const double e = -x * cosh(s) + lncosh(5.0 * s / 3.0);
        const double half = j ? 1.0 : 0.5;
        const double tK = exp(e) * half;
        sK += tK;
        sF += exp(e - lncosh(s)) * half;
        if (s > s_peak && tK <= 1e-19 * sK) break;
    }
    F = x * kH * sF;
    K = kH * sK;
}

// Ntail(x) = int_x^inf F(t)/t dt
__device__ double number_tail(double x) {
    const double s_peak = asinh(2.0 / (3.0 * x)) + 1.0;
    double sum = 0.0;
    for (int j = 0; j < 200000; ++j) {
        const double s = j * kH;
        const double e = -x * cosh(s) + lncosh(5.0 * s / 3.0) - 2.0 * lncosh(s);
        const double t = exp(e) * (j ? 1.0 : 0.5);
        sum += t;
        if (s > s_peak && t <= 1e-19 * sum) break;
    }
    return kH * sum;
}

// Node value y = L(t) and slope dL/dt of the F table at t = log2 x.
//   lower: L = log2 F - t/3,        dL/dt = 2/3 - x^2 K / F
//   upper: L = log2 F - t/3 + x log2 e, dL/dt = 2/3 - x^2 K / F + x
// (x F'/F = 1 - x^2 K_{5/3}/F since F' = F/x - x K_{5/3}).
__device__ void f_node(double t, bool upper, double &y, double &dy) {
    const double x = exp2(t);
    double F, K;
    synch_FK(x, F, K);
    y = log2(F) - t / 3.0;
    dy = 2.0 / 3.0 - x * x * K / F;
    if (upper) {
        y += x * 1.4426950408889634;
        dy += x;
    }
}

__device__ float4 hermite_piece(double y0, double d0, double y1, double d1, double h) {
    const double m0 = h * d0, m1 = h * d1;
    return make_float4((float)y0, (float)m0, (float)(3.0 * (y1 - y0) - 2.0 * m0 - m1),
                       (float)(2.0 * (y0 - y1) + m0 + m1));
}

__global__ void build_f_table(float4 *out) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= kFTotal) return;
    const bool upper = p >= kFLoN;
    const int j = upper ? (p - kFLoN + kFUpJ0) : (p + kFLoJ0);
    const double h = 1.0 / kFPerUnit;
    double y0, d0, y1, d1;
    f_node(j * h, upper, y0, d0);
    f_node((j + 1) * h, upper, y1, d1);
    out[p] = hermite_piece(y0, d0, y1, d1, h);
}

// Node of the trial-density table: y = log2 q, q = F(x)/(x S(x)), and dy/darg.
//   lower (arg u = log2 R', x = 2^{3u/4}, x S = (4/3) R'):
//       y = log2(3/4) + log2 F - u,           dy/du = (3/4)(1 - x^2 K/F) - 1
//   upper (arg v = -log2(1-R'), x = v ln2 - ln(9/7), S = 1 - R' = 2^{-v}):
//       y = log2 F - log2 x + v,              dy/dv = 1 - x K/F
// (x F'/F = 1 - x^2 K_{5/3}/F as above).
__device__ void g_node(double arg, bool upper, double &y, double &dy) {
    double x, F, K;
    if (!upper) {
        x = exp2(0.75 * arg);
        synch_FK(x, F, K);
        y = log2(0.75) + log2(F) - arg;
        dy = 0.75 * (1.0 - x * x * K / F) - 1.0;
    } else {
        x = arg * 0.69314718055994531 - log(9.0 / 7.0);
        synch_FK(x, F, K);
        y = log2(F) - log2(x) + arg;
        dy = 1.0 - x * K / F;
    }
}

__global__ void build_g_table(float4 *out) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= kGTotal) return;
    const bool upper = p >= kGLoN;
    const int j = upper ? (p - kGLoN + kGUpJ0) : (p + kGLoJ0);
    const double h = 1.0 / kGPerUnit;
    double y0, d0, y1, d1;
    g_node(j * h, upper, y0, d0);
    g_node((j + 1) * h, upper, y1, d1);
    out[p] = hermite_piece(y0, d0, y1, d1, h);
}

// K_{2/3}(xi), K_{1/3}(xi) and int_xi^inf K_{1/3} for the quantum kernel table,
// from K_nu(xi) = int_0^inf exp(-xi cosh s) cosh(nu s) ds and
// int_xi^inf K_nu = int_0^inf exp(-xi cosh s) cosh(nu s) / cosh s ds.
__device__ void bessel_triple(double xi, double &k23, double &k13, double &ki13) {
    const double s_peak = asinh(2.0 / (3.0 * xi)) + 1.0;
    double a = 0.0, b = 0.0, c = 0.0;
    for (int j = 0; j < 200000; ++j) {
        const double s = j * kH;
        const double e = -xi * cosh(s);
        const double half = j ? 1.0 : 0.5;
        const double ta = exp(e + lncosh(2.0 * s / 3.0)) * half;
        const double l13 = e + lncosh(s / 3.0);
        a += ta;
        b += exp(l13) * half;
        c += exp(l13 - lncosh(s)) * half;
        // the nu = 1/3 integrands fall faster than the nu = 2/3 one past the peak
        if (s > s_peak && ta <= 1e-19 * a) break;
    }
    k23 = kH * a;
    k13 = kH * b;
    ki13 = kH * c;
}

// Nodes of the quantum table at t = log2 xi (see kQPerUnit): values and
// d/dt, from K'_{2/3} = -K_{1/3} - (2/3) K_{2/3} / xi and (int_xi K_{1/3})' = -K_{1/3}:
//   dyA/dt = xi - xi K_{1/3}/K_{2/3},  dyB/dt = xi - xi K_{1/3} / int_xi K_{1/3}.
__device__ void q_node(double t, double &ya, double &da, double &yb, double &db) {
    const double xi = exp2(t);
    double k23, k13, ki13;
    bessel_triple(xi, k23, k13, ki13);
    const double xl = xi * 1.4426950408889634;
    ya = log2(k23) + 2.0 * t / 3.0 + xl;
    da = xi - xi * k13 / k23;
    yb = log2(ki13) + xl;
    db = xi - xi * k13 / ki13;
}

__global__ void build_q_table(float4 *out) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= kQN) return;
    const int j = p + kQJ0;
    const double h = 1.0 / kQPerUnit;
    double a0, da0, b0, db0, a1, da1, b1, db1;
    q_node(j * h, a0, da0, b0, db0);
    q_node((j + 1) * h, a1, da1, b1, db1);
    out[2 * p] = hermite_piece(a0, da0, a1, da1, h);
    out[2 * p + 1] = hermite_piece(b0, db0, b1, db1, h);
}

// x with N(x) = U N(inf), given U and 1-U (both accurate); bisection in log2 x.
__device__ double inv_number(double one_minus_u) {
    const double target = one_minus_u * kNInf;   // = Ntail(x)
    double lo = -100.0, hi = 8.0;                 // log2 x bracket
    for (int it = 0; it < 200; ++it) {
        const double mid = 0.5 * (lo + hi);
        if (mid <= lo || mid >= hi) break;
        if (number_tail(exp2(mid)) > target) lo = mid; else hi = mid;
    }
    return exp2(0.5 * (lo + hi));
}

// T1 node at logit w: y = log2 x, dy/dw = U (1-U) N(inf) / (ln2 F(x)).
__device__ void t1_node(double w, double &y, double &dy) {
    const double U = 1.0 / (1.0 + exp(-w));
    const double V = 1.0 / (1.0 + exp(w));       // 1 - U
    const double x = inv_number(V);
    double F, K;
    synch_FK(x, F, K);
    y = log2(x);
    dy = U * V * kNInf / (0.69314718055994531 * F);
}

__global__ void build_t1_table(float4 *out) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= kT1N) return;
    const double h = 2.0 * kT1W / kT1N;
    double y0, d0, y1, d1;
    t1_node(-kT1W + p * h, y0, d0);
    t1_node(-kT1W + (p + 1) * h, y1, d1);
    out[p] = hermite_piece(y0, d0, y1, d1, h);
}

// r(chi) = N(2/(3 chi)) / N(inf) and 1 - r on log10 chi nodes.
__global__ void build_r_table(float2 *out) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= kRN) return;
    const double chi = exp10(kRLogChiLo + (double)p / kRPerDecade);
    const double tail = number_tail(2.0 / (3.0 * chi)) / kNInf;
    out[p] = make_float2((float)(1.0 - tail), (float)tail);
}

// Root a of a^{4/3} + (7/9) e^{-a} = 1 (normalisation of S(x)), by Newton.
__global__ void solve_proposal(double *out) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    double a = 0.7;
    for (int it = 0; it < 60; ++it) {
        const double g = pow(a, 4.0 / 3.0) + (7.0 / 9.0) * exp(-a) - 1.0;
        const double dg = (4.0 / 3.0) * cbrt(a) - (7.0 / 9.0) * exp(-a);
        const double an = a - g / dg;
        if (an == a) break;
        a = an;
    }
    out[0] = a;
    out[1] = (double)(float)pow(a, 4.0 / 3.0);
}

// ---------------------------------------------------------------- evaluation
__global__ void eval_F_kernel(const float4 *__restrict__ tab, const float *__restrict__ x,
                              float *__restrict__ out, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float xv = x[i];
    if (!(xv > 0.0f)) { out[i] = 0.0f; return; }
    const float t = __log2f(xv);
    // branch point of the table families at x = 1 (both cover it)
    float L;
    if (t < 0.0f) {
        L = ftab_eval(tab, t, kFLoJ0, kFLoN, 0);
        out[i] = exp2f(L + t * (1.0f / 3.0f));
    } else {
        L = ftab_eval(tab, t, kFUpJ0, kFUpN, kFLoN);
        out[i] = exp2f(L + t * (1.0f / 3.0f) - xv * 1.4426950408889634f);
    }
}

__global__ void eval_trial_kernel(const float4 *__restrict__ gtab, float pa,
                                  const uint32_t *__restrict__ a, const float *__restrict__ rate,
                                  const float *__restrict__ chi, int kin_cut,
                                  float *__restrict__ dn, float *__restrict__ xo, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    float lg;
    bool lower;
    float d = rate[i] * trial_q(a[i], gtab, pa, lg, lower);
    if (trial_is_cut(trial_cut(kin_cut != 0, chi[i]), lg, lower)) d = 0.0f;
    dn[i] = d;
    xo[i] = trial_x(a[i], lg, lower);
}

__global__ void eval_quantum_kernel(const float4 *__restrict__ qtab, float pa,
                                    const uint32_t *__restrict__ a, const float *__restrict__ rate,
                                    const float *__restrict__ chi, float *__restrict__ dn,
                                    float *__restrict__ xo, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    float x;
    dn[i] = rate[i] * quantum_q(a[i], qtab, pa, chi[i], x);
    xo[i] = x;
}

__global__ void philox_kernel(const uint4 *__restrict__ ctr, uint32_t k0, uint32_t k1,
                              uint4 *__restrict__ out, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    out[i] = philox4x32_10(ctr[i], k0, k1);
}

}  // namespace
}  // namespace sr

using namespace sr;

extern "C" int sr_table_build(sr_table **out, void *stream) {
    if (!out) return SR_E_INVAL;
    *out = nullptr;
    hipStream_t st = (hipStream_t)stream;
    sr_table *t = new (std::nothrow) sr_table();
    if (!t) return SR_E_NOMEM;
    double *aux = nullptr;
    auto fail = [&](int code) {
        if (t->ftab) (void)hipFree(t->ftab);
        if (t->gtab) (void)hipFree(t->gtab);
        if (t->qtab) (void)hipFree(t->qtab);
        if (t->t1) (void)hipFree(t->t1);
        if (t->r) (void)hipFree(t->r);
        if (aux) (void)hipFree(aux);
        delete t;
        return code;
    };
    if (hipGetDevice(&t->device) != hipSuccess) return fail(SR_E_HIP);
    if (hipMalloc(&t->ftab, sizeof(float4) * kFTotal) != hipSuccess) return fail(SR_E_NOMEM);
    if (hipMalloc(&t->gtab, sizeof(float4) * kGTotal) != hipSuccess) return fail(SR_E_NOMEM);
    if (hipMalloc(&t->qtab, sizeof(float4) * 2 * kQN) != hipSuccess) return fail(SR_E_NOMEM);
    if (hipMalloc(&t->t1, sizeof(float4) * kT1N) != hipSuccess) return fail(SR_E_NOMEM);
    if (hipMalloc(&t->r, sizeof(float2) * kRN) != hipSuccess) return fail(SR_E_NOMEM);
    if (hipMalloc(&aux, sizeof(double) * 2) != hipSuccess) return fail(SR_E_NOMEM);
    build_f_table<<<(kFTotal + 63) / 64, 64, 0, st>>>(t->ftab);
    build_g_table<<<(kGTotal + 63) / 64, 64, 0, st>>>(t->gtab);
    build_q_table<<<(kQN + 63) / 64, 64, 0, st>>>(t->qtab);
    build_t1_table<<<(kT1N + 63) / 64, 64, 0, st>>>(t->t1);
    build_r_table<<<(kRN + 63) / 64, 64, 0, st>>>(t->r);
    solve_proposal<<<1, 64, 0, st>>>(aux);
    if (hipGetLastError() != hipSuccess) return fail(SR_E_HIP);
    double host[2];
    if (hipMemcpyAsync(host, aux, sizeof host, hipMemcpyDeviceToHost, st) != hipSuccess)
        return fail(SR_E_HIP);
    if (hipStreamSynchronize(st) != hipSuccess) return fail(SR_E_HIP);
    (void)hipFree(aux);
    aux = nullptr;
    t->a = host[0];
    t->pa = (float)host[1];
    *out = t;
    return SR_OK;
}

extern "C" void sr_table_free(sr_table *t) {
    if (!t) return;
    if (t->ftab) (void)hipFree(t->ftab);
    if (t->gtab) (void)hipFree(t->gtab);
    if (t->qtab) (void)hipFree(t->qtab);
    if (t->t1) (void)hipFree(t->t1);
    if (t->r) (void)hipFree(t->r);
    delete t;
}

extern "C" int sr_table_query(const sr_table *t, sr_table_info *info) {
    if (!t || !info) return SR_E_INVAL;
    info->proposal_pa = t->pa;
    info->f_pieces = kFTotal;
    info->g_pieces = kGTotal;
    info->q_pieces = kQN;
    info->proposal_a = t->a;
    info->t1_pieces = kT1N;
    info->r_nodes = kRN;
    info->r_log10chi_lo = kRLogChiLo;
    info->r_log10chi_hi = kRLogChiHi;
    return SR_OK;
}

extern "C" int sr_eval_synchrotron_F(const sr_table *t, const float *x, float *out, int64_t n,
                                     void *stream) {
    if (!t || n < 0 || (n > 0 && (!x || !out))) return SR_E_INVAL;
    if (n == 0) return SR_OK;
    eval_F_kernel<<<(unsigned)((n + 255) / 256), 256, 0, (hipStream_t)stream>>>(t->ftab, x, out, n);
    SR_HIP_CHECK(hipGetLastError());
    return SR_OK;
}

extern "C" int sr_eval_trial(const sr_table *t, const uint32_t *a, const float *rate,
                             const float *chi, int32_t kin_cut, float *out_dn, float *out_x,
                             int64_t n, void *stream) {
    if (!t || n < 0 || (n > 0 && (!a || !rate || !chi || !out_dn || !out_x))) return SR_E_INVAL;
    if (n == 0) return SR_OK;
    eval_trial_kernel<<<(unsigned)((n + 255) / 256), 256, 0, (hipStream_t)stream>>>(
        t->gtab, t->pa, a, rate, chi, kin_cut, out_dn, out_x, n);
    SR_HIP_CHECK(hipGetLastError());
    return SR_OK;
}

extern "C" int sr_eval_trial_quantum(const sr_table *t, const uint32_t *a, const float *rate,
                                     const float *chi, float *out_dn, float *out_x, int64_t n,
                                     void *stream) {
    if (!t || n < 0 || (n > 0 && (!a || !rate || !chi || !out_dn || !out_x))) return SR_E_INVAL;
    if (n == 0) return SR_OK;
    eval_quantum_kernel<<<(unsigned)((n + 255) / 256), 256, 0, (hipStream_t)stream>>>(
        t->qtab, t->pa, a, rate, chi, out_dn, out_x, n);
    SR_HIP_CHECK(hipGetLastError());
    return SR_OK;
}

extern "C" int sr_philox(const uint32_t *ctr, uint64_t seed, uint32_t *out, int64_t n,
                         void *stream) {
    if (n < 0 || (n > 0 && (!ctr || !out))) return SR_E_INVAL;
    if (n == 0) return SR_OK;
    philox_kernel<<<(unsigned)((n + 255) / 256), 256, 0, (hipStream_t)stream>>>(
        (const uint4 *)ctr, (uint32_t)seed, (uint32_t)(seed >> 32), (uint4 *)out, n);
    SR_HIP_CHECK(hipGetLastError());
    return SR_OK;
}
