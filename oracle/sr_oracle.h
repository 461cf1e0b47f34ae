/*
 * sr_oracle.h -- plain FP64 CPU oracle for the real-time synchrotron emission
 * method of Wallin, Gonoskov & Marklund (arXiv 1409.5574).
 *
 * TEST INFRASTRUCTURE ONLY.  This library exists to check the GPU path.  Only
 * the test suite, the smoke check and the CPU-baseline leg of the benchmark may
 * load it.  It shares no code, header, table or constant generator with the
 * HIP library under paper_1409_5574_amd/csrc.
 *
 * Normalised units throughout: c = m = e = 1, electron charge q = -1, time in
 * 1/omega_r, momentum in mc, energy in mc^2, fields eE/(mc omega_r),
 * eB/(m omega_r).
 */
#ifndef SR_ORACLE_H
#define SR_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Philox4x32 with 10 rounds (Salmon, Moraes, Dror & Shaw, SC'11). */
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);
void orc_philox_array(int64_t n, const uint32_t *ctr, const uint32_t key[2], uint32_t *out);

/* Synchrotron function F(x) = x * int_x^inf K_{5/3}(t) dt (section "Modelling
 * the relativistic case", equation after eq:synchrotron).  Trapezoid rule on
 * the integral representation x * int_0^inf exp(-x cosh s) cosh(5s/3)/cosh s ds
 * with step h (0 < h); h <= 0 selects the default 0.1. */
double orc_synchrotron_F(double x, double h);
void orc_synchrotron_F_array(int64_t n, const double *x, double *out, double h);

/* Proposal S(x) (section "Monte Carlo method"): root a of a^{4/3} + (7/9)e^{-a} = 1. */
double orc_proposal_a(void);
/* Branch threshold P(a) = a^{4/3}, rounded to the nearest binary32 value. */
double orc_proposal_Pa_f32(void);
/* Inverse of P at R': x and S(x) from the branch chosen by R' <= Pa. */
void orc_proposal_invert(double Rp, double Pa, double *x, double *S);

/* dN of one trial (steps 3-5 of the recipe): rate * F(x)/(x S(x)), zero for x > xcut. */
double orc_trial_dn(double Rp, double Pa, double rate, double xcut, double *x_out);

/* Relativistic Boris push for charge q: p -> p_new. */
void orc_boris(const double p[3], const double E[3], const double B[3], double q,
               double dt, double p_new[3]);

/* Effective magnetic field (eq:effective_H) with the limiter dp_perp/p <= 1.
 * Returns H_eff; writes the mean gamma and the (unclamped) ratio dp_perp/p. */
double orc_heff(const double p_old[3], const double p_new[3], double dt,
                double *gamma_bar, double *ratio);

enum { ORC_FIELD_ANALYTIC = 0, ORC_FIELD_2D = 2, ORC_FIELD_3D = 3 };
enum { ORC_RECOIL_NONE = 0, ORC_RECOIL_PHOTON = 1, ORC_RECOIL_LL = 2 };
enum { ORC_DN_WEIGHT = 0, ORC_DN_CLAMP = 1 };
/* ORC_SAMPLER_S: the proposal S(x) and F(x)/x; ORC_SAMPLER_DIRECT: total rate
 * and the inverse number CDF; ORC_SAMPLER_QUANTUM: the proposal S(x) with the
 * quantum kernel Q(x, chi) below (kin_cut is implied by Q). */
enum { ORC_SAMPLER_S = 0, ORC_SAMPLER_DIRECT = 1, ORC_SAMPLER_QUANTUM = 2 };
/* Modified Bessel function K_nu(xi) = int_0^inf exp(-xi cosh s) cosh(nu s) ds
 * and its tail int_xi^inf K_nu = int_0^inf exp(-xi cosh s) cosh(nu s)/cosh s ds,
 * by the trapezoid rule with step h (h <= 0: 0.1). */
double orc_bessel_K(double nu, double xi, double h);
double orc_bessel_K_tail(double nu, double xi, double h);
/* Quantum-corrected emission kernel (reading for chi approaching 1, section
 * "Limitations"; the quantum synchrotron spectrum of Baier-Katkov / Ritus):
 * with delta = 1.5 chi x and xi = x/(1-delta),
 *   Q(x, chi) = (1 - delta + 1/(1-delta)) K_{2/3}(xi) - int_xi^inf K_{1/3},
 * zero for delta >= 1; dN/(dt dx) = (sqrt3/2pi) alpha H_eff Q, and
 * Q(x, 0) = F(x)/x. */
double orc_quantum_kernel(double x, double chi, double h);
void orc_quantum_kernel_array(int64_t n, const double *x, const double *chi, double *out, double h);
/* dN of one quantum trial: rate * Q(x, chi) / S(x) at the proposal's x(R'). */
double orc_trial_dn_quantum(double Rp, double Pa, double rate, double chi, double *x_out);

typedef struct {
    int32_t kind;          /* ORC_FIELD_* */
    int64_t n[3];          /* cells per axis (2D: n[2] ignored) */
    double dx[3];
    double origin[3];
    double e0[3], b0[3];   /* uniform fields for ORC_FIELD_ANALYTIC */
    const float *E[3];     /* Yee-staggered component arrays, x fastest */
    const float *B[3];
} orc_field;

typedef struct {
    double hbar_n;         /* hbar omega_r / (m c^2) */
    double alpha;          /* fine-structure constant */
    int32_t n_samples;     /* K frequency trials per particle and step */
    int32_t recoil;        /* ORC_RECOIL_* */
    int32_t dn_policy;     /* ORC_DN_* */
    int32_t kin_cut;       /* 1: reject x > 2/(3 chi) */
    int32_t sampler;       /* ORC_SAMPLER_* */
    int32_t push_position; /* 1: advance positions */
    double omega_grid;     /* > 0: the grid's cutoff frequency c/dx (section "The
                              field setup"); photons of lower frequency are not
                              emitted as particles (the grid carries them).
                              0: no floor */
} orc_params;

/* Photons in id order, then sample order.  Capacity must be >= n*K. */
typedef struct {
    int64_t capacity;
    int64_t count;
    double *eps, *w;
    double *dir;     /* [capacity][3] */
    double *pos;     /* [capacity][3] */
    uint32_t *parent, *k;
} orc_photons;

/* E and B at a position (uniform values, or CIC on the Yee grid). */
void orc_gather(const orc_field *f, const double pos[3], double E[3], double B[3]);

/* Optional per-particle / per-sample diagnostics (any pointer may be NULL). */
typedef struct {
    double *heff, *gamma_bar, *chi, *ratio;      /* [n] */
    double *dn, *xs, *rp;                        /* [n*K] */
    uint32_t *bword;                             /* [n*K] */
    uint8_t *emit;                               /* [n*K] */
} orc_detail;

/* Number spectrum with the kinematic cut (direct sampler).
 * orc_number_integral(x) = int_0^x F(t)/t dt, by the trapezoid rule on
 * int_0^inf cosh(5s/3) (1 - exp(-x cosh s)) / cosh^2 s ds; x = +inf gives 5 pi/3.
 * orc_energy_integral(x) = int_0^x F(t) dt, likewise.
 * orc_inv_number_cdf: x with int_0^x F/t = u * int_0^xmax F/t, xmax = 2/(3 chi)
 * when kin_cut, else unbounded; bisection in log x to FP64 resolution. */
double orc_number_integral(double x, double h);
double orc_energy_integral(double x, double h);
double orc_inv_number_cdf(double chi, double u, int32_t kin_cut);

/* One time step for n particles.  State arrays are FP64 and updated in place
 * (x,y,z may be NULL when positions are not used).  ledger[5] receives
 * {emitted, LL loss, recoil dE, clamped, dropped}.  Returns 0, or -1 on a bad
 * argument, -2 if the photon capacity is too small. */
int orc_step(int64_t n, double *x, double *y, double *z,
             double *px, double *py, double *pz, const double *w, const uint32_t *id,
             const orc_field *f, double dt, uint64_t seed, uint64_t step,
             const orc_params *prm,
             orc_photons *ph, double ledger[5], orc_detail *det, int32_t threads);

/* Closing the PIC loop: charge and current on the Yee grid (see the C file
 * for units).  CIC charge on the nodes, rho[i + nx (j + ny k)] += q w S / dV. */
int orc_deposit_rho(int64_t n, const double *x, const double *y, const double *z,
                    const double *w, double q, int32_t dim, const int64_t nn[3],
                    const double dx[3], double *rho);
/* Esirkepov charge-conserving current of the moves x0 -> x1 (each below one
 * cell, taken the shorter way round the periodic box); vz: the z velocity for
 * 2D (ignored in 3D).  Adds into jx, jy, jz.  Returns 0, -1 on a bad argument,
 * -2 on a move of a cell or more. */
int orc_deposit_current(int64_t n, const double *x0, const double *y0, const double *z0,
                        const double *x1, const double *y1, const double *z1, const double *vz,
                        const double *w, double q, double dt, int32_t dim, const int64_t nn[3],
                        const double dx[3], double *jx, double *jy, double *jz);
#ifdef __cplusplus
}
#endif
#endif
