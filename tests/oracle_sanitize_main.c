/*
 * oracle_sanitize_main.c -- drives every entry point of the C oracle on small
 * inputs, for a host build with AddressSanitizer and UndefinedBehaviorSanitizer
 * (tests/test_oracle_sanitize.py).  Test infrastructure: it exercises the
 * oracle's memory accesses and integer/float conversions, including its edge
 * cases (particles at rest, a non-finite field value, positions outside the
 * box, moves across the periodic boundary, a photon buffer of exactly n K
 * slots), and prints "ok" when every call returned its expected code.
 */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "sr_oracle.h"

static uint64_t lcg_state = 0x9E3779B97F4A7C15ull;
static double urand(void)
{
    lcg_state = lcg_state * 6364136223846793005ull + 1442695040888963407ull;
    return (double)(lcg_state >> 11) * 0x1p-53;
}

static int fail(const char *what, int code)
{
    fprintf(stderr, "FAIL %s: %d\n", what, code);
    return 1;
}

/* one orc_step over n particles of a field, with every diagnostic array */
static int run_step(const char *label, const orc_field *f, int dim, int64_t n, int K, int sampler,
                    int recoil, int dn_policy, int kin_cut, double p_scale, double omega_grid)
{
    double *x = malloc(sizeof(double) * n), *y = malloc(sizeof(double) * n);
    double *z = malloc(sizeof(double) * n);
    double *px = malloc(sizeof(double) * n), *py = malloc(sizeof(double) * n);
    double *pz = malloc(sizeof(double) * n), *w = malloc(sizeof(double) * n);
    uint32_t *id = malloc(sizeof(uint32_t) * n);
    const int64_t cap = n * K;
    orc_photons ph;
    ph.capacity = cap;
    ph.count = 0;
    ph.eps = malloc(sizeof(double) * cap);
    ph.w = malloc(sizeof(double) * cap);
    ph.dir = malloc(sizeof(double) * 3 * cap);
    ph.pos = malloc(sizeof(double) * 3 * cap);
    ph.parent = malloc(sizeof(uint32_t) * cap);
    ph.k = malloc(sizeof(uint32_t) * cap);
    orc_detail det;
    det.heff = malloc(sizeof(double) * n);
    det.gamma_bar = malloc(sizeof(double) * n);
    det.chi = malloc(sizeof(double) * n);
    det.ratio = malloc(sizeof(double) * n);
    det.dn = malloc(sizeof(double) * cap);
    det.xs = malloc(sizeof(double) * cap);
    det.rp = malloc(sizeof(double) * cap);
    det.bword = malloc(sizeof(uint32_t) * cap);
    det.emit = malloc(cap);
    const double L[3] = {f->n[0] * f->dx[0], f->n[1] * f->dx[1], f->n[2] * f->dx[2]};
    for (int64_t i = 0; i < n; ++i) {
        /* some positions outside the box on either side, some on its edges */
        x[i] = (1.4 * urand() - 0.2) * (dim ? L[0] : 1.0);
        y[i] = (1.4 * urand() - 0.2) * (dim ? L[1] : 1.0);
        z[i] = (1.4 * urand() - 0.2) * (dim == 3 ? L[2] : 1.0);
        if (i % 11 == 0) x[i] = 0.0;
        if (i % 13 == 0 && dim) y[i] = L[1];
        px[i] = p_scale * (2.0 * urand() - 1.0);
        py[i] = p_scale * (2.0 * urand() - 1.0);
        pz[i] = p_scale * (2.0 * urand() - 1.0);
        if (i % 7 == 0) px[i] = py[i] = pz[i] = 0.0;   /* at rest */
        w[i] = 0.5 + urand();
        id[i] = (uint32_t)(i * 2654435761u);
    }
    orc_params prm;
    memset(&prm, 0, sizeof(prm));
    prm.hbar_n = 1e-4;
    prm.alpha = 1.0 / 137.035999;
    prm.n_samples = K;
    prm.recoil = recoil;
    prm.dn_policy = dn_policy;
    prm.kin_cut = kin_cut;
    prm.sampler = sampler;
    prm.push_position = 1;
    prm.omega_grid = omega_grid;
    double led[5];
    const int rc = orc_step(n, dim ? x : NULL, dim ? y : NULL, dim == 3 ? z : NULL, px, py, pz, w,
                            id, f, 0.05, 7, 3, &prm, &ph, led, &det, 1);
    int bad = rc != 0 || ph.count < 0 || ph.count > cap;
    for (int c = 0; c < 5 && !bad; ++c) bad = isnan(led[c]);
    printf("%s: rc %d, %lld photons, emitted %.6e\n", label, rc, (long long)ph.count, led[0]);
    /* too small a photon buffer */
    ph.capacity = cap - 1;
    if (orc_step(n, x, y, z, px, py, pz, w, id, f, 0.05, 7, 4, &prm, &ph, led, NULL, 1) != -2)
        bad = 1;
    free(x); free(y); free(z); free(px); free(py); free(pz); free(w); free(id);
    free(ph.eps); free(ph.w); free(ph.dir); free(ph.pos); free(ph.parent); free(ph.k);
    free(det.heff); free(det.gamma_bar); free(det.chi); free(det.ratio); free(det.dn);
    free(det.xs); free(det.rp); free(det.bword); free(det.emit);
    return bad ? fail(label, rc) : 0;
}

static float *grid_component(int64_t cells, double amp)
{
    float *a = malloc(sizeof(float) * cells);
    for (int64_t i = 0; i < cells; ++i) a[i] = (float)(amp * (2.0 * urand() - 1.0));
    return a;
}

static int run_deposits(int dim)
{
    const int64_t nn[3] = {5, 4, dim == 3 ? 3 : 1};
    const double dx[3] = {0.25, 0.3, 0.2};
    const int64_t cells = nn[0] * nn[1] * nn[2];
    const int64_t n = 300;
    double *x0 = malloc(sizeof(double) * n), *y0 = malloc(sizeof(double) * n);
    double *z0 = malloc(sizeof(double) * n), *x1 = malloc(sizeof(double) * n);
    double *y1 = malloc(sizeof(double) * n), *z1 = malloc(sizeof(double) * n);
    double *vz = malloc(sizeof(double) * n), *w = malloc(sizeof(double) * n);
    double *rho = calloc(cells, sizeof(double));
    double *jx = calloc(cells, sizeof(double)), *jy = calloc(cells, sizeof(double));
    double *jz = calloc(cells, sizeof(double));
    const double L[3] = {nn[0] * dx[0], nn[1] * dx[1], nn[2] * dx[2]};
    for (int64_t i = 0; i < n; ++i) {
        double *p0[3] = {x0, y0, z0}, *p1[3] = {x1, y1, z1};
        for (int a = 0; a < 3; ++a) {
            p0[a][i] = urand() * L[a];
            double v = p0[a][i] + (1.9 * urand() - 0.95) * dx[a];   /* below a cell */
            if (v < 0.0) v += L[a];                                  /* across the boundary */
            if (v >= L[a]) v -= L[a];
            p1[a][i] = v;
        }
        vz[i] = 2.0 * urand() - 1.0;
        w[i] = urand();
    }
    int bad = orc_deposit_rho(n, x0, y0, z0, w, -1.0, dim, nn, dx, rho) != 0;
    bad |= orc_deposit_current(n, x0, y0, z0, x1, y1, z1, vz, w, -1.0, 0.1, dim, nn, dx, jx, jy,
                               jz) != 0;
    /* a move of more than a cell is refused */
    x1[0] = x0[0] + 1.5 * dx[0];
    if (x1[0] >= L[0]) x1[0] -= L[0];
    bad |= orc_deposit_current(n, x0, y0, z0, x1, y1, z1, vz, w, -1.0, 0.1, dim, nn, dx, jx, jy,
                               jz) != -2;
    free(x0); free(y0); free(z0); free(x1); free(y1); free(z1); free(vz); free(w);
    free(rho); free(jx); free(jy); free(jz);
    printf("deposits %dD: %s\n", dim, bad ? "bad" : "ok");
    return bad ? fail("deposits", dim) : 0;
}

int main(void)
{
    int bad = 0;

    uint32_t ctr[12], out[12];
    const uint32_t key[2] = {0xDEADBEEFu, 0x12345678u};
    for (int i = 0; i < 12; ++i) ctr[i] = (uint32_t)(i * 0x01000193u);
    orc_philox_array(3, ctr, key, out);

    const double xs[4] = {1e-6, 0.3, 2.0, 25.0};
    double F[4];
    orc_synchrotron_F_array(4, xs, F, 0.0);
    double chi_arr[4] = {1e-3, 0.1, 1.0, 5.0}, Q[4];
    orc_quantum_kernel_array(4, xs, chi_arr, Q, 0.0);
    for (int i = 0; i < 4; ++i) bad |= !(isfinite(F[i]) && isfinite(Q[i]));
    bad |= !isfinite(orc_number_integral(INFINITY, 0.0));
    bad |= !isfinite(orc_energy_integral(3.0, 0.0));
    bad |= !isfinite(orc_inv_number_cdf(0.5, 0.999, 1));
    bad |= !isfinite(orc_inv_number_cdf(1e-5, 1e-7, 0));
    const double Pa = orc_proposal_Pa_f32();
    double xo, So;
    orc_proposal_invert(0.5 * Pa, Pa, &xo, &So);
    orc_proposal_invert(1.0 - 0x1p-24, Pa, &xo, &So);
    bad |= !isfinite(orc_trial_dn(0.1, Pa, 0.3, 4.0, &xo));
    bad |= !isfinite(orc_trial_dn_quantum(0.9, Pa, 0.3, 2.0, &xo));
    bad |= !isfinite(orc_bessel_K(2.0 / 3.0, 0.01, 0.0)) || !isfinite(orc_bessel_K_tail(1.0 / 3.0, 8.0, 0.0));
    const double p0[3] = {0.0, 0.0, 0.0}, E[3] = {1.0, -2.0, 0.5}, B[3] = {0.0, 3.0, 40.0};
    double p1[3], gb, ratio;
    orc_boris(p0, E, B, -1.0, 0.05, p1);
    bad |= !isfinite(orc_heff(p0, p0, 0.05, &gb, &ratio));   /* at rest */
    bad |= !isfinite(orc_heff(p0, p1, 0.05, &gb, &ratio));
    if (bad) return fail("special functions", 0);

    /* uniform fields */
    orc_field fa;
    memset(&fa, 0, sizeof(fa));
    fa.kind = ORC_FIELD_ANALYTIC;
    fa.n[0] = fa.n[1] = fa.n[2] = 1;
    fa.dx[0] = fa.dx[1] = fa.dx[2] = 1.0;
    fa.b0[0] = 0.3; fa.b0[2] = 40.0;
    bad |= run_step("uniform S weight photon", &fa, 0, 64, 8, ORC_SAMPLER_S, ORC_RECOIL_PHOTON,
                    ORC_DN_WEIGHT, 1, 2000.0, 0.0);
    bad |= run_step("uniform S clamp LL", &fa, 0, 64, 3, ORC_SAMPLER_S, ORC_RECOIL_LL, ORC_DN_CLAMP,
                    0, 2000.0, 0.0);
    bad |= run_step("uniform direct", &fa, 0, 48, 2, ORC_SAMPLER_DIRECT, ORC_RECOIL_NONE,
                    ORC_DN_WEIGHT, 1, 500.0, 0.0);
    bad |= run_step("uniform quantum", &fa, 0, 48, 4, ORC_SAMPLER_QUANTUM, ORC_RECOIL_PHOTON,
                    ORC_DN_WEIGHT, 1, 5e5, 0.0);

    /* 2D grid of 5 x 4 cells, one component holding a NaN */
    orc_field f2;
    memset(&f2, 0, sizeof(f2));
    f2.kind = ORC_FIELD_2D;
    f2.n[0] = 5; f2.n[1] = 4; f2.n[2] = 1;
    f2.dx[0] = 0.2; f2.dx[1] = 0.25; f2.dx[2] = 1.0;
    float *c2[6];
    for (int c = 0; c < 6; ++c) c2[c] = grid_component(20, 50.0);
    c2[1][7] = NAN;
    for (int c = 0; c < 3; ++c) { f2.E[c] = c2[c]; f2.B[c] = c2[3 + c]; }
    bad |= run_step("2D S grid floor", &f2, 2, 200, 4, ORC_SAMPLER_S, ORC_RECOIL_PHOTON,
                    ORC_DN_WEIGHT, 1, 300.0, 1e-3);
    bad |= run_step("2D direct", &f2, 2, 100, 1, ORC_SAMPLER_DIRECT, ORC_RECOIL_LL, ORC_DN_CLAMP,
                    1, 300.0, 0.0);

    /* 3D grid of 4 x 3 x 5 cells, one component holding an infinity */
    orc_field f3;
    memset(&f3, 0, sizeof(f3));
    f3.kind = ORC_FIELD_3D;
    f3.n[0] = 4; f3.n[1] = 3; f3.n[2] = 5;
    f3.dx[0] = 0.2; f3.dx[1] = 0.25; f3.dx[2] = 0.3;
    float *c3[6];
    for (int c = 0; c < 6; ++c) c3[c] = grid_component(60, 80.0);
    c3[5][13] = INFINITY;
    for (int c = 0; c < 3; ++c) { f3.E[c] = c3[c]; f3.B[c] = c3[3 + c]; }
    bad |= run_step("3D S", &f3, 3, 256, 8, ORC_SAMPLER_S, ORC_RECOIL_PHOTON, ORC_DN_WEIGHT, 1,
                    3000.0, 0.0);
    bad |= run_step("3D quantum floor", &f3, 3, 128, 2, ORC_SAMPLER_QUANTUM, ORC_RECOIL_PHOTON,
                    ORC_DN_CLAMP, 1, 3e5, 1e-2);
    for (int c = 0; c < 6; ++c) { free(c2[c]); free(c3[c]); }

    bad |= run_deposits(2);
    bad |= run_deposits(3);

    if (bad) return 1;
    printf("ok\n");
    return 0;
}
