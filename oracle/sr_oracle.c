/*
 * sr_oracle.c -- plain FP64 CPU oracle for the real-time synchrotron photon
 * emission method of Wallin, Gonoskov & Marklund (arXiv 1409.5574).
 *
 * TEST INFRASTRUCTURE ONLY: loaded by the test suite, the smoke check and the
 * CPU-baseline leg of the benchmark, never by the product path.  Written from
 * the paper's equations; it shares nothing with the HIP library.
 *
 * Every function below follows one passage of the paper (named in its
 * comment) or, where the paper is silent, the reading stated beside it.  No
 * blocking, caching or reordering beyond what the definitions state: each
 * particle is processed on its own, samples in order, in FP64.
 *
 * Normalised units: c = m = e = 1, q = -1 for the electron; time 1/omega_r,
 * momentum mc, energy mc^2.
 */
#include "sr_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* ------------------------------------------------------------------------ */
/* Philox4x32-10, from the published definition (Salmon et al., SC'11):      */
/* ten rounds of two 32x32->64 multiplies; the key is bumped by the Weyl     */
/* constants between rounds.                                                 */
/* ------------------------------------------------------------------------ */
static void philox_round(uint32_t c[4], const uint32_t k[2])
{
    const uint64_t prod0 = (uint64_t)0xD2511F53u * (uint64_t)c[0];
    const uint64_t prod1 = (uint64_t)0xCD9E8D57u * (uint64_t)c[2];
    const uint32_t hi0 = (uint32_t)(prod0 >> 32), lo0 = (uint32_t)prod0;
    const uint32_t hi1 = (uint32_t)(prod1 >> 32), lo1 = (uint32_t)prod1;
    const uint32_t n0 = hi1 ^ c[1] ^ k[0];
    const uint32_t n1 = lo1;
    const uint32_t n2 = hi0 ^ c[3] ^ k[1];
    const uint32_t n3 = lo0;
    c[0] = n0; c[1] = n1; c[2] = n2; c[3] = n3;
}

void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    uint32_t c[4] = {ctr[0], ctr[1], ctr[2], ctr[3]};
    uint32_t k[2] = {key[0], key[1]};
    for (int r = 0; r < 10; ++r) {
        if (r > 0) {
            k[0] += 0x9E3779B9u;
            k[1] += 0xBB67AE85u;
        }
        philox_round(c, k);
    }
    memcpy(out, c, sizeof c);
}

/* ------------------------------------------------------------------------ */
/* Synchrotron function (section "Modelling the relativistic case"):         */
/*   F(x) = x int_x^inf K_{5/3}(t) dt.                                        */
/* With K_nu(t) = int_0^inf exp(-t cosh s) cosh(nu s) ds, the t-integral is  */
/* done in closed form:                                                      */
/*   F(x) = x int_0^inf exp(-x cosh s) cosh(5s/3) / cosh s ds.               */
/* The integrand is even and analytic in |Im s| < pi/2, so the trapezoid     */
/* rule converges like exp(-pi^2/h).                                         */
/* ------------------------------------------------------------------------ */
static double log_cosh(double y)
{
    y = fabs(y);
    return y + log1p(exp(-2.0 * y)) - M_LN2;
}

double orc_synchrotron_F(double x, double h)
{
    if (!(x > 0.0)) return 0.0;
    if (h <= 0.0) h = 0.1;
    /* the integrand peaks near sinh s = 2/(3x); stop well past it */
    const double s_peak = asinh(2.0 / (3.0 * x));
    double sum = 0.0;
    for (long j = 0; j < 2000000; ++j) {
        const double s = j * h;
        const double e = -x * cosh(s) + log_cosh(5.0 * s / 3.0) - log_cosh(s);
        const double term = exp(e) * (j == 0 ? 0.5 : 1.0);
        sum += term;
        if (s > s_peak && term <= 1e-20 * sum) break;
    }
    return x * h * sum;
}

void orc_synchrotron_F_array(int64_t n, const double *x, double *out, double h)
{
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t i = 0; i < n; ++i) out[i] = orc_synchrotron_F(x[i], h);
}

/* int_0^x F(t)/t dt = int_0^inf cosh(5s/3) (1 - exp(-x cosh s)) / cosh^2 s ds */
double orc_number_integral(double x, double h)
{
    if (!(x > 0.0)) return 0.0;
    if (h <= 0.0) h = 0.1;
    double sum = 0.0;
    for (long j = 0; j < 2000000; ++j) {
        const double s = j * h;
        const double c = cosh(s);
        const double one_minus = isinf(x) ? 1.0 : -expm1(-x * c);
        const double lw = log_cosh(5.0 * s / 3.0) - 2.0 * log_cosh(s);
        const double term = exp(lw) * one_minus * (j == 0 ? 0.5 : 1.0);
        sum += term;
        /* integrand decays like exp(-s/3); its tail beyond s is ~3x the term */
        if (s > 1.0 && 3.0 * term / h <= 1e-18 * sum) break;
    }
    return h * sum;
}

/* 1 - (1+y) e^{-y}, accurate for small y */
static double one_minus_1py_emy(double y)
{
    if (y < 0.1) {
        /* sum_{k>=2} (-1)^k (k-1) y^k / k! */
        double term = y * y / 2.0; /* k = 2: (1) y^2/2! */
        double fact_pow = y * y / 2.0; /* y^k/k! */
        double sum = 0.0;
        for (int k = 2; k < 40; ++k) {
            term = ((k & 1) ? -1.0 : 1.0) * (double)(k - 1) * fact_pow;
            sum += term;
            fact_pow *= y / (double)(k + 1);
            if (fabs(term) < 1e-30 * fabs(sum)) break;
        }
        return sum;
    }
    return 1.0 - (1.0 + y) * exp(-y);
}

/* int_0^x F(t) dt = int_0^inf cosh(5s/3) [1 - (1 + x c) e^{-x c}] / c^3 ds, c = cosh s */
double orc_energy_integral(double x, double h)
{
    if (!(x > 0.0)) return 0.0;
    if (h <= 0.0) h = 0.1;
    double sum = 0.0;
    for (long j = 0; j < 2000000; ++j) {
        const double s = j * h;
        const double c = cosh(s);
        const double g = isinf(x) ? 1.0 : one_minus_1py_emy(x * c);
        const double lw = log_cosh(5.0 * s / 3.0) - 3.0 * log_cosh(s);
        const double term = exp(lw) * g * (j == 0 ? 0.5 : 1.0);
        sum += term;
        if (s > 1.0 && term / h <= 1e-19 * sum) break;
    }
    return h * sum;
}

double orc_inv_number_cdf(double chi, double u, int32_t kin_cut)
{
    const double xmax = (kin_cut && chi > 0.0) ? 2.0 / (3.0 * chi) : INFINITY;
    const double total = orc_number_integral(xmax, 0.0);
    const double target = u * total;
    double lo = log(1e-40);
    double hi = isinf(xmax) ? log(1e3) : log(xmax);
    for (int it = 0; it < 400; ++it) {
        const double mid = 0.5 * (lo + hi);
        if (mid == lo || mid == hi) break;
        if (orc_number_integral(exp(mid), 0.0) < target) lo = mid; else hi = mid;
    }
    return exp(0.5 * (lo + hi));
}

/* ------------------------------------------------------------------------ */
/* Proposal density S(x) (section "Monte Carlo method"):                     */
/*   S = (4/3) x^{1/3} for x < a,  (7/9) e^{-x} for x > a,  int S = 1.        */
/* P(x) = x^{4/3} below a and 1 - (7/9) e^{-x} above, so                      */
/*   lower: x = R'^{3/4}, S = (4/3) R'^{1/4};  upper: x = -ln((9/7)(1-R')),    */
/*   S = 1 - R'.                                                             */
/* ------------------------------------------------------------------------ */
double orc_proposal_a(void)
{
    double lo = 0.5, hi = 1.0; /* g(0.5) < 0 < g(1) */
    for (int it = 0; it < 200; ++it) {
        const double mid = 0.5 * (lo + hi);
        if (mid == lo || mid == hi) break;
        const double g = pow(mid, 4.0 / 3.0) + (7.0 / 9.0) * exp(-mid) - 1.0;
        if (g < 0.0) lo = mid; else hi = mid;
    }
    return 0.5 * (lo + hi);
}

double orc_proposal_Pa_f32(void)
{
    return (double)(float)pow(orc_proposal_a(), 4.0 / 3.0);
}

void orc_proposal_invert(double Rp, double Pa, double *x, double *S)
{
    if (Rp <= Pa) {
        *x = pow(Rp, 0.75);
        *S = (4.0 / 3.0) * pow(Rp, 0.25);
    } else {
        *x = -log((9.0 / 7.0) * (1.0 - Rp));
        *S = 1.0 - Rp;
    }
}

/* Steps 3-5 of the recipe for one trial: frequency from R', proposal value,
 * and dN = rate F(x) / (x S(x)) with rate = dt (sqrt3/2pi) alpha H_eff; zero
 * above the kinematic cut xcut. */
double orc_trial_dn(double Rp, double Pa, double rate, double xcut, double *x_out)
{
    double x, S;
    orc_proposal_invert(Rp, Pa, &x, &S);
    if (x_out) *x_out = x;
    if (x > xcut) return 0.0;
    return rate * orc_synchrotron_F(x, 0.0) / (x * S);
}

/* ------------------------------------------------------------------------ */
/* Quantum-corrected spectrum for chi approaching 1 (section "Limitations":   */
/* the classical expression fails there and a QED treatment is needed; the   */
/* paper gives no formula).  Reading: the quantum synchrotron spectrum of    */
/* Baier & Katkov / Ritus, written in the method's variable x = omega/omega_c */
/* with delta = hbar omega / (gamma m c^2) = 1.5 chi x and xi = x / (1-delta): */
/*   dN/(dt dx) = (sqrt3/2pi) alpha H_eff Q(x, chi),                          */
/*   Q = (1 - delta + 1/(1-delta)) K_{2/3}(xi) - int_xi^inf K_{1/3}(t) dt,    */
/* and Q = 0 for delta >= 1 (no photon above the emitter's energy).  As      */
/* chi -> 0, Q -> 2 K_{2/3}(x) - int_x^inf K_{1/3} = int_x^inf K_{5/3} =      */
/* F(x)/x, the classical kernel of the method.                               */
/* ------------------------------------------------------------------------ */

/* K_nu(xi) = int_0^inf exp(-xi cosh s) cosh(nu s) ds (entire integrand: the  */
/* trapezoid rule converges faster than any power of h).                      */
double orc_bessel_K(double nu, double xi, double h)
{
    if (!(xi > 0.0)) return INFINITY;
    if (h <= 0.0) h = 0.1;
    const double s_peak = asinh(fabs(nu) / xi);
    double sum = 0.0;
    for (long j = 0; j < 2000000; ++j) {
        const double s = j * h;
        const double term = exp(-xi * cosh(s) + log_cosh(nu * s)) * (j == 0 ? 0.5 : 1.0);
        sum += term;
        if (s > s_peak && term <= 1e-20 * sum) break;
    }
    return h * sum;
}

/* int_xi^inf K_nu(t) dt = int_0^inf exp(-xi cosh s) cosh(nu s) / cosh s ds  */
/* (the t-integral of the representation above done in closed form).         */
double orc_bessel_K_tail(double nu, double xi, double h)
{
    if (!(xi > 0.0)) return INFINITY;
    if (h <= 0.0) h = 0.1;
    const double s_peak = asinh(fabs(nu) / xi) + 1.0;
    double sum = 0.0;
    for (long j = 0; j < 2000000; ++j) {
        const double s = j * h;
        const double term = exp(-xi * cosh(s) + log_cosh(nu * s) - log_cosh(s)) *
                            (j == 0 ? 0.5 : 1.0);
        sum += term;
        if (s > s_peak && term <= 1e-20 * sum) break;
    }
    return h * sum;
}

double orc_quantum_kernel(double x, double chi, double h)
{
    if (!(x > 0.0)) return 0.0;
    const double delta = 1.5 * chi * x;
    if (!(delta < 1.0)) return 0.0;
    const double om = 1.0 - delta;
    const double xi = x / om;
    return (om + 1.0 / om) * orc_bessel_K(2.0 / 3.0, xi, h) - orc_bessel_K_tail(1.0 / 3.0, xi, h);
}

void orc_quantum_kernel_array(int64_t n, const double *x, const double *chi, double *out, double h)
{
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t i = 0; i < n; ++i) out[i] = orc_quantum_kernel(x[i], chi[i], h);
}

/* One trial of the quantum sampler: the proposal of the classical method with */
/* the quantum kernel in place of F(x)/x, so dN = rate x Q / (x S) = rate Q / S. */
double orc_trial_dn_quantum(double Rp, double Pa, double rate, double chi, double *x_out)
{
    double x, S;
    orc_proposal_invert(Rp, Pa, &x, &S);
    if (x_out) *x_out = x;
    return rate * orc_quantum_kernel(x, chi, 0.0) / S;
}

/* ------------------------------------------------------------------------ */
/* Boris push (the scheme the section "Numerical implementation" describes:  */
/* half electric kick, magnetic rotation, half electric kick).               */
/* ------------------------------------------------------------------------ */
void orc_boris(const double p[3], const double E[3], const double B[3], double q,
               double dt, double p_new[3])
{
    const double h = 0.5 * q * dt;
    double um[3], t[3], s[3], up[3], upl[3];
    for (int c = 0; c < 3; ++c) um[c] = p[c] + h * E[c];
    const double g = sqrt(1.0 + um[0] * um[0] + um[1] * um[1] + um[2] * um[2]);
    for (int c = 0; c < 3; ++c) t[c] = h * B[c] / g;
    const double t2 = t[0] * t[0] + t[1] * t[1] + t[2] * t[2];
    for (int c = 0; c < 3; ++c) s[c] = 2.0 * t[c] / (1.0 + t2);
    up[0] = um[0] + (um[1] * t[2] - um[2] * t[1]);
    up[1] = um[1] + (um[2] * t[0] - um[0] * t[2]);
    up[2] = um[2] + (um[0] * t[1] - um[1] * t[0]);
    upl[0] = um[0] + (up[1] * s[2] - up[2] * s[1]);
    upl[1] = um[1] + (up[2] * s[0] - up[0] * s[2]);
    upl[2] = um[2] + (up[0] * s[1] - up[1] * s[0]);
    for (int c = 0; c < 3; ++c) p_new[c] = upl[c] + h * E[c];
}

static double gamma_of(const double p[3])
{
    return sqrt(1.0 + p[0] * p[0] + p[1] * p[1] + p[2] * p[2]);
}

/* ------------------------------------------------------------------------ */
/* Effective magnetic field, eq:effective_H, with the momentum the average   */
/* of the two neighbouring steps and the limiter dp_perp/p <= 1 (same        */
/* section).  gamma is taken as the mean of the two gammas.                  */
/* ------------------------------------------------------------------------ */
double orc_heff(const double p_old[3], const double p_new[3], double dt,
                double *gamma_bar, double *ratio)
{
    double pb[3], d[3];
    for (int c = 0; c < 3; ++c) {
        pb[c] = 0.5 * (p_old[c] + p_new[c]);
        d[c] = p_new[c] - p_old[c];
    }
    const double gb = 0.5 * (gamma_of(p_old) + gamma_of(p_new));
    if (gamma_bar) *gamma_bar = gb;
    const double p2 = pb[0] * pb[0] + pb[1] * pb[1] + pb[2] * pb[2];
    if (!(p2 > 0.0)) {
        if (ratio) *ratio = 0.0;
        return 0.0;
    }
    const double d2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
    const double pd = pb[0] * d[0] + pb[1] * d[1] + pb[2] * d[2];
    double num = p2 * d2 - pd * pd;
    if (num < 0.0) num = 0.0;
    const double r = sqrt(num) / p2;
    if (ratio) *ratio = r;
    return gb * (r < 1.0 ? r : 1.0) / dt;
}

/* ------------------------------------------------------------------------ */
/* Field gather: cloud-in-cell on a Yee grid, periodic.  Component offsets   */
/* in cells: Ex(1/2,0,0) Ey(0,1/2,0) Ez(0,0,1/2) Bx(0,1/2,1/2) By(1/2,0,1/2)  */
/* Bz(1/2,1/2,0).  Values are the FP32 grid values widened to FP64.          */
/* ------------------------------------------------------------------------ */
static const double yee_off[6][3] = {
    {0.5, 0.0, 0.0}, {0.0, 0.5, 0.0}, {0.0, 0.0, 0.5},
    {0.0, 0.5, 0.5}, {0.5, 0.0, 0.5}, {0.5, 0.5, 0.0},
};

static int64_t wrap_index(int64_t i, int64_t n)
{
    int64_t r = i % n;
    return r < 0 ? r + n : r;
}

static double cic_component(const orc_field *f, const float *arr, const double off[3],
                            const double pos[3])
{
    const int dims = (f->kind == ORC_FIELD_3D) ? 3 : 2;
    int64_t i0[3] = {0, 0, 0};
    double fr[3] = {0.0, 0.0, 0.0};
    for (int a = 0; a < dims; ++a) {
        const double u = (pos[a] - f->origin[a]) / f->dx[a] - off[a];
        const double fl = floor(u);
        i0[a] = (int64_t)fl;
        fr[a] = u - fl;
    }
    const int64_t nx = f->n[0], ny = f->n[1];
    const int nzc = (dims == 3) ? 2 : 1;
    double val = 0.0;
    for (int dz = 0; dz < nzc; ++dz) {
        const int64_t kk = (dims == 3) ? wrap_index(i0[2] + dz, f->n[2]) : 0;
        const double wz = (dims == 3) ? (dz ? fr[2] : 1.0 - fr[2]) : 1.0;
        for (int dy = 0; dy < 2; ++dy) {
            const int64_t jj = wrap_index(i0[1] + dy, ny);
            const double wy = dy ? fr[1] : 1.0 - fr[1];
            for (int dxi = 0; dxi < 2; ++dxi) {
                const int64_t ii = wrap_index(i0[0] + dxi, nx);
                const double wx = dxi ? fr[0] : 1.0 - fr[0];
                val += wx * wy * wz * (double)arr[ii + nx * (jj + ny * kk)];
            }
        }
    }
    return val;
}

void orc_gather(const orc_field *f, const double pos[3], double E[3], double B[3])
{
    if (f->kind == ORC_FIELD_ANALYTIC) {
        for (int c = 0; c < 3; ++c) { E[c] = f->e0[c]; B[c] = f->b0[c]; }
        return;
    }
    for (int c = 0; c < 3; ++c) {
        E[c] = cic_component(f, f->E[c], yee_off[c], pos);
        B[c] = cic_component(f, f->B[c], yee_off[3 + c], pos);
    }
}

/* ------------------------------------------------------------------------ */
/* One step of the emission method for one particle (the six steps listed at */
/* the end of section "Monte Carlo method", preceded by the push).           */
/* ------------------------------------------------------------------------ */
typedef struct {
    double led[5];
    int nph;
} particle_result;

static const double TWO_POW_M23 = 1.0 / 8388608.0;
static const double TWO_POW_32 = 4294967296.0;

static void step_one(int64_t i, double *x, double *y, double *z,
                     double *px, double *py, double *pz, const double *w, const uint32_t *id,
                     const orc_field *f, double dt, uint64_t seed, uint64_t step,
                     const orc_params *prm, double Pa,
                     /* per-particle photon slots [K] */
                     double *s_eps, double *s_w, double *s_dir, double *s_pos, uint8_t *s_on,
                     particle_result *res, orc_detail *det)
{
    const int K = prm->n_samples;
    const double wi = w[i];
    double pos[3] = {x ? x[i] : 0.0, y ? y[i] : 0.0, z ? z[i] : 0.0};
    const double p_old[3] = {px[i], py[i], pz[i]};
    double E[3], B[3], p_new[3];

    orc_gather(f, pos, E, B);
    orc_boris(p_old, E, B, -1.0, dt, p_new);

    /* steps 1-2: H_eff (limited), then omega_c = 1.5 H gamma^2 and chi */
    double gb = 0.0, ratio = 0.0;
    double H = orc_heff(p_old, p_new, dt, &gb, &ratio);
    /* The paper assumes finite fields and momenta.  A particle whose push is not
       finite (a non-finite field value or momentum) is given H_eff = chi = 0:
       it emits nothing and adds nothing to the ledger, and its momentum and
       position are stored as computed. */
    const int bad = !(isfinite(p_new[0]) && isfinite(p_new[1]) && isfinite(p_new[2]) &&
                      isfinite(H) && isfinite(gb));
    if (bad) H = 0.0;
    const double chi = bad ? 0.0 : prm->hbar_n * H * gb;
    double pbar[3], pbm;
    for (int c = 0; c < 3; ++c) pbar[c] = 0.5 * (p_old[c] + p_new[c]);
    pbm = sqrt(pbar[0] * pbar[0] + pbar[1] * pbar[1] + pbar[2] * pbar[2]);
    double dir[3] = {0.0, 0.0, 0.0};
    if (pbm > 0.0) for (int c = 0; c < 3; ++c) dir[c] = pbar[c] / pbm;

    if (det) {
        if (det->heff) det->heff[i] = H;
        if (det->gamma_bar) det->gamma_bar[i] = gb;
        if (det->chi) det->chi[i] = chi;
        if (det->ratio) det->ratio[i] = ratio;
    }

    /* d N = dt (sqrt3/2pi) alpha H F(x) / (x S(x)) per trial (reading of the
       emission-count formula with x = omega/omega_c) */
    const double rate = dt * (sqrt(3.0) / (2.0 * M_PI)) * prm->alpha * H;
    const double xcut = (prm->kin_cut && chi > 0.0) ? 2.0 / (3.0 * chi) : INFINITY;
    double direct_W = 0.0;
    if (prm->sampler == ORC_SAMPLER_DIRECT && H > 0.0)
        direct_W = rate * orc_number_integral(xcut, 0.0);

    const uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    double emitted = 0.0, delta = 0.0;
    res->nph = 0;
    uint32_t words[4] = {0, 0, 0, 0};
    for (int k = 0; k < K; ++k) {
        if ((k & 1) == 0) {
            const uint32_t ctr[4] = {id[i], (uint32_t)step, (uint32_t)(k >> 1), 0u};
            orc_philox4x32_10(ctr, key, words);
        }
        const uint32_t a = words[2 * (k & 1)];
        const uint32_t b = words[2 * (k & 1) + 1];
        /* step 3: uniform R' as a 23-bit midpoint, never 0 or 1 */
        const double Rp = ((double)(a >> 9) + 0.5) * TWO_POW_M23;
        double xs = 0.0, dN = 0.0;
        if (prm->sampler == ORC_SAMPLER_S) {
            dN = orc_trial_dn(Rp, Pa, rate, xcut, &xs);         /* steps 3-5 */
        } else if (prm->sampler == ORC_SAMPLER_QUANTUM) {
            dN = orc_trial_dn_quantum(Rp, Pa, rate, chi, &xs);  /* steps 3-5, quantum kernel */
        } else {
            dN = direct_W;
        }
        /* step 6: compare with the second uniform at 32-bit resolution */
        int emit;
        double frac; /* photon weight / particle weight */
        if (dN >= 1.0) {
            emit = 1;
            frac = (prm->dn_policy == ORC_DN_WEIGHT) ? dN / K : 1.0 / K;
        } else {
            emit = ((double)b < floor(dN * TWO_POW_32));
            frac = 1.0 / K;
        }
        if (emit && prm->sampler == ORC_SAMPLER_DIRECT)
            xs = orc_inv_number_cdf(chi, Rp, prm->kin_cut);
        /* grid cutoff: a photon below omega_grid (hbar omega_c x < hbar omega_grid)
           is resolved by the grid and is not emitted as a particle */
        if (emit && prm->omega_grid > 0.0 && 1.5 * chi * gb * xs < prm->hbar_n * prm->omega_grid)
            emit = 0;
        if (det) {
            const int64_t s = i * K + k;
            if (det->dn) det->dn[s] = dN;
            if (det->xs) det->xs[s] = xs;
            if (det->rp) det->rp[s] = Rp;
            if (det->bword) det->bword[s] = b;
            if (det->emit) det->emit[s] = (uint8_t)emit;
        }
        s_on[k] = (uint8_t)emit;
        if (emit) {
            const double eps = 1.5 * chi * gb * xs; /* hbar omega_c x */
            s_eps[k] = eps;
            s_w[k] = wi * frac;
            for (int c = 0; c < 3; ++c) {
                s_dir[3 * k + c] = dir[c];
                s_pos[3 * k + c] = pos[c];
            }
            emitted += wi * frac * eps;
            delta += frac * eps;
            res->nph++;
        }
    }

    /* Landau-Lifshitz loss (eq:LLformOfRRForce): |f.v| dt = (2/3)(alpha/hbar_n) chi^2 beta^2 dt */
    const double beta2 = (gb > 0.0) ? (pbm * pbm) / (gb * gb) : 0.0;
    const double ll = bad ? 0.0 : wi * (2.0 / 3.0) * (prm->alpha / prm->hbar_n) * chi * chi * beta2 * dt;

    /* recoil: reduce |p| along the post-push momentum */
    double clamped = 0.0, dE = 0.0;
    if (prm->recoil == ORC_RECOIL_LL && !bad)
        delta = dt * (2.0 / 3.0) * (prm->alpha / prm->hbar_n) * chi * chi * (gb > 0.0 ? pbm / gb : 0.0);
    else if (prm->recoil == ORC_RECOIL_NONE)
        delta = 0.0;
    if (delta > 0.0) {
        const double pm = sqrt(p_new[0] * p_new[0] + p_new[1] * p_new[1] + p_new[2] * p_new[2]);
        const double g_before = gamma_of(p_new);
        double fac = (pm > 0.0) ? 1.0 - delta / pm : 0.0;
        if (fac < 0.0) {
            clamped = wi * (delta - pm);
            fac = 0.0;
        }
        for (int c = 0; c < 3; ++c) p_new[c] *= fac;
        dE = wi * (gamma_of(p_new) - g_before);
    }

    px[i] = p_new[0]; py[i] = p_new[1]; pz[i] = p_new[2];

    if (prm->push_position) {
        const double g = gamma_of(p_new);
        double *xyz[3] = {x, y, z};
        const int dims = (f->kind == ORC_FIELD_3D) ? 3 : (f->kind == ORC_FIELD_2D ? 2 : 3);
        for (int a = 0; a < dims; ++a) {
            if (!xyz[a]) continue;
            double v = pos[a] + dt * p_new[a] / g;
            if (f->kind != ORC_FIELD_ANALYTIC) {
                const double L = f->n[a] * f->dx[a];
                v -= L * floor((v - f->origin[a]) / L);
                if (v - f->origin[a] >= L) v -= L; /* guard against rounding to L */
            }
            xyz[a][i] = v;
        }
    }

    res->led[0] = emitted;
    res->led[1] = ll;
    res->led[2] = dE;
    res->led[3] = clamped;
    res->led[4] = 0.0;
}

int orc_step(int64_t n, double *x, double *y, double *z,
             double *px, double *py, double *pz, const double *w, const uint32_t *id,
             const orc_field *f, double dt, uint64_t seed, uint64_t step,
             const orc_params *prm,
             orc_photons *ph, double ledger[5], orc_detail *det, int32_t threads)
{
    if (n < 0 || !px || !py || !pz || !w || !id || !f || !prm || !ph || !ledger) return -1;
    const int K = prm->n_samples;
    if (K < 1) return -1;
    if (ph->capacity < n * (int64_t)K) return -2;
    const double Pa = orc_proposal_Pa_f32();

    double *s_eps = (double *)malloc(sizeof(double) * (size_t)(n * K + 1));
    double *s_w = (double *)malloc(sizeof(double) * (size_t)(n * K + 1));
    double *s_dir = (double *)malloc(sizeof(double) * 3 * (size_t)(n * K + 1));
    double *s_pos = (double *)malloc(sizeof(double) * 3 * (size_t)(n * K + 1));
    uint8_t *s_on = (uint8_t *)malloc((size_t)(n * K + 1));
    particle_result *res = (particle_result *)malloc(sizeof(particle_result) * (size_t)(n + 1));
    if (!s_eps || !s_w || !s_dir || !s_pos || !s_on || !res) {
        free(s_eps); free(s_w); free(s_dir); free(s_pos); free(s_on); free(res);
        return -1;
    }
#ifdef _OPENMP
    if (threads > 0) omp_set_num_threads(threads);
#else
    (void)threads;
#endif

#pragma omp parallel for schedule(dynamic, 256)
    for (int64_t i = 0; i < n; ++i)
        step_one(i, x, y, z, px, py, pz, w, id, f, dt, seed, step, prm, Pa,
                 s_eps + i * K, s_w + i * K, s_dir + 3 * i * K, s_pos + 3 * i * K, s_on + i * K,
                 res + i, det);

    /* photons in particle order then sample order; ledger Kahan-summed in order */
    int64_t cnt = 0;
    double sum[5] = {0, 0, 0, 0, 0}, comp[5] = {0, 0, 0, 0, 0};
    for (int64_t i = 0; i < n; ++i) {
        for (int k = 0; k < K; ++k) {
            const int64_t s = i * K + k;
            if (!s_on[s]) continue;
            ph->eps[cnt] = s_eps[s];
            ph->w[cnt] = s_w[s];
            for (int c = 0; c < 3; ++c) {
                ph->dir[3 * cnt + c] = s_dir[3 * s + c];
                ph->pos[3 * cnt + c] = s_pos[3 * s + c];
            }
            ph->parent[cnt] = id[i];
            ph->k[cnt] = (uint32_t)k;
            ++cnt;
        }
        for (int c = 0; c < 5; ++c) {
            const double yv = res[i].led[c] - comp[c];
            const double t = sum[c] + yv;
            comp[c] = (t - sum[c]) - yv;
            sum[c] = t;
        }
    }
    ph->count = cnt;
    for (int c = 0; c < 5; ++c) ledger[c] = sum[c];

    free(s_eps); free(s_w); free(s_dir); free(s_pos); free(s_on); free(res);
    return 0;
}

/* Array helper for tests: n independent Philox4x32-10 blocks. */
void orc_philox_array(int64_t n, const uint32_t *ctr, const uint32_t key[2], uint32_t *out)
{
    for (int64_t i = 0; i < n; ++i) orc_philox4x32_10(ctr + 4 * i, key, out + 4 * i);
}

/* ------------------------------------------------------------------------ */
/* Closing the PIC loop (the field solve and current deposition of the PIC  */
/* codes the method runs in: section "The field setup" -- particles on a    */
/* grid with Maxwell's equations, the currents feeding the grid).           */
/*                                                                          */
/* Normalised units: E, B in m c omega_r / e, lengths in c / omega_r,       */
/* densities in n_r = m omega_r^2 / (4 pi e^2), so div E = rho and          */
/* dE/dt = curl B - J.  A macro-particle of weight w carries charge q w in  */
/* units of n_r (c/omega_r)^3; rho and J are per cell volume dV.            */
/*                                                                          */
/* Charge: first-order (cloud-in-cell) shape on the nodes (i, j, k).        */
/* Current: Esirkepov's charge-conserving decomposition of the change of    */
/* that shape between x^n and x^{n+1} (Comput. Phys. Commun. 135, 144,      */
/* 2001), Jx at (i+1/2, j, k), Jy at (i, j+1/2, k), Jz at (i, j, k+1/2); in */
/* 2D (no z dependence) Jz sits on the nodes and carries q w v_z.           */
/* ------------------------------------------------------------------------ */

/* CIC weights of coordinate u (in cells) on the four nodes base..base+3. */
static void shape4(double u, int64_t base, double s[4])
{
    for (int a = 0; a < 4; ++a) {
        const double d = fabs(u - (double)(base + a));
        s[a] = d < 1.0 ? 1.0 - d : 0.0;
    }
}

int orc_deposit_rho(int64_t n, const double *x, const double *y, const double *z,
                    const double *w, double q, int32_t dim, const int64_t nn[3],
                    const double dx[3], double *rho)
{
    if (n < 0 || !x || !y || !w || !rho || (dim != 2 && dim != 3) || (dim == 3 && !z)) return -1;
    const int64_t nx = nn[0], ny = nn[1], nz = dim == 3 ? nn[2] : 1;
    const double dV = dx[0] * dx[1] * (dim == 3 ? dx[2] : 1.0);
    for (int64_t p = 0; p < n; ++p) {
        const double u[3] = {x[p] / dx[0], y[p] / dx[1], dim == 3 ? z[p] / dx[2] : 0.0};
        int64_t b[3];
        double s[3][4];
        for (int a = 0; a < 3; ++a) {
            b[a] = (int64_t)floor(u[a]) - 1;
            shape4(u[a], b[a], s[a]);
        }
        const int kz = dim == 3 ? 4 : 1;
        for (int c = 0; c < kz; ++c)
            for (int bj = 0; bj < 4; ++bj)
                for (int ai = 0; ai < 4; ++ai) {
                    const double wt = s[0][ai] * s[1][bj] * (dim == 3 ? s[2][c] : 1.0);
                    if (wt == 0.0) continue;
                    const int64_t i = wrap_index(b[0] + ai, nx), j = wrap_index(b[1] + bj, ny);
                    const int64_t k = dim == 3 ? wrap_index(b[2] + c, nz) : 0;
                    rho[i + nx * (j + ny * k)] += q * w[p] * wt / dV;
                }
    }
    return 0;
}

/* The displacement x1 - x0 is taken modulo the box (the shorter way round) and
 * must be below one cell on every axis; returns -2 otherwise. */
int orc_deposit_current(int64_t n, const double *x0, const double *y0, const double *z0,
                        const double *x1, const double *y1, const double *z1, const double *vz,
                        const double *w, double q, double dt, int32_t dim, const int64_t nn[3],
                        const double dx[3], double *jx, double *jy, double *jz)
{
    if (n < 0 || !x0 || !y0 || !x1 || !y1 || !w || !jx || !jy || !jz || !(dt > 0.0)) return -1;
    if (dim != 2 && dim != 3) return -1;
    if (dim == 3 && (!z0 || !z1)) return -1;
    if (dim == 2 && !vz) return -1;
    const int64_t nx = nn[0], ny = nn[1], nz = dim == 3 ? nn[2] : 1;
    const double dV = dx[0] * dx[1] * (dim == 3 ? dx[2] : 1.0);
    const int64_t ncell[3] = {nx, ny, nz};
    for (int64_t p = 0; p < n; ++p) {
        const double a0[3] = {x0[p], y0[p], dim == 3 ? z0[p] : 0.0};
        const double a1[3] = {x1[p], y1[p], dim == 3 ? z1[p] : 0.0};
        double u0[3], u1[3];
        int64_t b[3];
        double S0[3][4], S1[3][4], D[3][4];
        const int na = dim;
        for (int a = 0; a < 3; ++a) {
            if (a >= na) { u0[a] = u1[a] = 0.0; b[a] = 0; continue; }
            const double L = (double)ncell[a] * dx[a];
            double d = a1[a] - a0[a];
            d -= L * floor(d / L + 0.5);           /* shorter way round the box */
            u0[a] = a0[a] / dx[a];
            u1[a] = u0[a] + d / dx[a];
            if (!(fabs(u1[a] - u0[a]) < 1.0)) return -2;
            b[a] = (int64_t)floor(u0[a]) - 1;
            shape4(u0[a], b[a], S0[a]);
            shape4(u1[a], b[a], S1[a]);
            for (int c = 0; c < 4; ++c) D[a][c] = S1[a][c] - S0[a][c];
        }
        const double qw = q * w[p];
        if (dim == 3) {
            /* Jx: W_x = Dx (S0y S0z + Dy S0z/2 + S0y Dz/2 + Dy Dz/3), summed along x */
            for (int c = 0; c < 4; ++c)
                for (int bj = 0; bj < 4; ++bj) {
                    double acc = 0.0;
                    const double fy = S0[1][bj] * S0[2][c] + 0.5 * D[1][bj] * S0[2][c] +
                                      0.5 * S0[1][bj] * D[2][c] + D[1][bj] * D[2][c] / 3.0;
                    for (int ai = 0; ai < 4; ++ai) {
                        acc -= qw * (dx[0] / dt) * D[0][ai] * fy / dV;
                        const int64_t i = wrap_index(b[0] + ai, nx), j = wrap_index(b[1] + bj, ny),
                                      k = wrap_index(b[2] + c, nz);
                        jx[i + nx * (j + ny * k)] += acc;
                    }
                }
            for (int c = 0; c < 4; ++c)
                for (int ai = 0; ai < 4; ++ai) {
                    double acc = 0.0;
                    const double fx = S0[0][ai] * S0[2][c] + 0.5 * D[0][ai] * S0[2][c] +
                                      0.5 * S0[0][ai] * D[2][c] + D[0][ai] * D[2][c] / 3.0;
                    for (int bj = 0; bj < 4; ++bj) {
                        acc -= qw * (dx[1] / dt) * D[1][bj] * fx / dV;
                        const int64_t i = wrap_index(b[0] + ai, nx), j = wrap_index(b[1] + bj, ny),
                                      k = wrap_index(b[2] + c, nz);
                        jy[i + nx * (j + ny * k)] += acc;
                    }
                }
            for (int bj = 0; bj < 4; ++bj)
                for (int ai = 0; ai < 4; ++ai) {
                    double acc = 0.0;
                    const double fz = S0[0][ai] * S0[1][bj] + 0.5 * D[0][ai] * S0[1][bj] +
                                      0.5 * S0[0][ai] * D[1][bj] + D[0][ai] * D[1][bj] / 3.0;
                    for (int c = 0; c < 4; ++c) {
                        acc -= qw * (dx[2] / dt) * D[2][c] * fz / dV;
                        const int64_t i = wrap_index(b[0] + ai, nx), j = wrap_index(b[1] + bj, ny),
                                      k = wrap_index(b[2] + c, nz);
                        jz[i + nx * (j + ny * k)] += acc;
                    }
                }
        } else {
            /* 2D: W_x = Dx (S0y + Dy/2), W_y = Dy (S0x + Dx/2); Jz = q w vz
               (S0x S0y + Dx S0y/2 + S0x Dy/2 + Dx Dy/3) / dV on the nodes */
            for (int bj = 0; bj < 4; ++bj) {
                double acc = 0.0;
                const double fy = S0[1][bj] + 0.5 * D[1][bj];
                for (int ai = 0; ai < 4; ++ai) {
                    acc -= qw * (dx[0] / dt) * D[0][ai] * fy / dV;
                    jx[wrap_index(b[0] + ai, nx) + nx * wrap_index(b[1] + bj, ny)] += acc;
                }
            }
            for (int ai = 0; ai < 4; ++ai) {
                double acc = 0.0;
                const double fx = S0[0][ai] + 0.5 * D[0][ai];
                for (int bj = 0; bj < 4; ++bj) {
                    acc -= qw * (dx[1] / dt) * D[1][bj] * fx / dV;
                    jy[wrap_index(b[0] + ai, nx) + nx * wrap_index(b[1] + bj, ny)] += acc;
                }
            }
            for (int bj = 0; bj < 4; ++bj)
                for (int ai = 0; ai < 4; ++ai) {
                    const double wt = S0[0][ai] * S0[1][bj] + 0.5 * D[0][ai] * S0[1][bj] +
                                      0.5 * S0[0][ai] * D[1][bj] + D[0][ai] * D[1][bj] / 3.0;
                    jz[wrap_index(b[0] + ai, nx) + nx * wrap_index(b[1] + bj, ny)] +=
                        qw * vz[p] * wt / dV;
                }
        }
    }
    return 0;
}

