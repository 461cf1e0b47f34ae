"""Pins of the oracle's quantum-corrected emission kernel Q(x, chi).

The paper states that its classical expression fails as chi approaches 1 and
that a QED treatment is needed there (section "Limitations"), without giving
one.  The oracle's reading is the quantum synchrotron spectrum of Baier-Katkov
/ Ritus, written in the method's variable x = omega/omega_c (delta = 1.5 chi x,
xi = x/(1 - delta)):

    Q(x, chi) = (1 - delta + 1/(1 - delta)) K_{2/3}(xi) - int_xi^inf K_{1/3},

zero for delta >= 1.  Each test checks the oracle against something that is not
the oracle: scipy's Bessel functions, the classical kernel, an independent
integral representation of the total rate and power (the Baier-Katkov form in
u = delta/(1 - delta), which uses K_{2/3} alone), the textbook small-chi
expansion of the radiated power, and brute-force quadrature of the estimator.
"""
import math

import numpy as np
import pytest
from scipy import integrate, special

import synth

SQ3 = math.sqrt(3.0)


@pytest.mark.parametrize("nu", [1 / 3, 2 / 3, 5 / 3])
@pytest.mark.parametrize("xi", [1e-6, 1e-3, 0.1, 1.0, 7.0, 60.0])
def test_bessel_K_matches_scipy(oracle, nu, xi):
    assert oracle.bessel_K(nu, xi) == pytest.approx(special.kv(nu, xi), rel=1e-12)


@pytest.mark.parametrize("xi", [1e-4, 0.01, 0.5, 2.0, 20.0])
def test_bessel_K_tail_matches_scipy_quadrature(oracle, xi):
    ref = integrate.quad(lambda t: special.kv(1 / 3, t), xi, np.inf, epsabs=0, epsrel=1e-12,
                         limit=400)[0]
    assert oracle.bessel_K_tail(1 / 3, xi) == pytest.approx(ref, rel=1e-9)


def test_bessel_K_tail_total_closed_form(oracle):
    # int_0^inf K_nu = pi / (2 cos(nu pi / 2)); for nu = 1/3 that is pi/sqrt3.  Near
    # 0, int_0^xi K_{1/3} ~ (3/4) Gamma(1/3) 2^{1/3} xi^{2/3} (from K_nu ~ Gamma(nu)/2 (2/t)^nu)
    xi = 1e-12
    head = 0.75 * special.gamma(1 / 3) * 2 ** (1 / 3) * xi ** (2 / 3)
    assert oracle.bessel_K_tail(1 / 3, xi) + head == pytest.approx(math.pi / SQ3, rel=1e-9)


@pytest.mark.parametrize("x", [1e-4, 0.01, 0.3, 2.0, 10.0])
def test_classical_limit_is_F_over_x(oracle, x):
    # 2 K_{2/3} - int K_{1/3} = int K_{5/3}: the quantum coefficient must tend to 2
    assert oracle.quantum_kernel(x, 1e-15)[0] == pytest.approx(
        oracle.synchrotron_F(x)[0] / x, rel=1e-12)


def test_kinematic_edge(oracle):
    chi = 0.7
    xe = 2 / (3 * chi)
    q = oracle.quantum_kernel([xe, xe * 1.0001, 5 * xe, xe * 0.99, xe * 0.9], chi)
    assert q[0] == 0.0 and q[1] == 0.0 and q[2] == 0.0
    # vanishes continuously at the edge (xi = x/(1-delta) -> inf), positive below it
    assert 0.0 < q[3] < 1e-30 < q[4]


def _x_integral(oracle, chi, power):
    """int_0^{2/(3chi)} x^power Q(x, chi) dx in t = ln x, plus the head below x0
    from Q ~ Gamma(2/3) 2^{2/3} x^{-2/3} (a 1e-30 head is far below the tolerance)."""
    xmax = 2 / (3 * chi)
    x0 = 1e-30

    def f(t):
        x = math.exp(t)
        return x ** (power + 1) * oracle.quantum_kernel(x, chi)[0]

    # split where the integrand changes character: small x, the peak, the edge
    pts = sorted({math.log(x0), math.log(min(1e-3, xmax / 10)), math.log(xmax / 2),
                  math.log(xmax * 0.9), math.log(xmax * 0.99), math.log(xmax)})
    tot = 0.0
    for a, b in zip(pts[:-1], pts[1:]):
        if b > a:
            tot += integrate.quad(f, a, b, epsabs=0, epsrel=1e-12, limit=400)[0]
    head = special.gamma(2 / 3) * 2 ** (2 / 3) * x0 ** (power + 1 / 3) / (power + 1 / 3)
    return tot + head


def _bk_integral(chi, poly, power):
    """int_0^inf poly(u) / (1+u)^power K_{2/3}(2u/(3chi)) du (scipy's K)."""
    f = lambda u: poly(u) / (1 + u) ** power * special.kv(2 / 3, 2 * u / (3 * chi))
    pts = [0.0, 1e-8, 1e-4 * chi, chi, 10 * chi, 100 * chi + 10]
    tot = 0.0
    for a, b in zip(pts[:-1], pts[1:]):
        tot += integrate.quad(f, a, b, epsabs=0, epsrel=1e-12, limit=400)[0]
    return tot + integrate.quad(f, pts[-1], np.inf, epsabs=0, epsrel=1e-12, limit=400)[0]


@pytest.mark.parametrize("chi", [0.05, 0.5, 2.0, 20.0])
def test_total_rate_matches_baier_katkov_form(oracle, chi):
    # int Q dx = 2/(9 chi) int_0^inf (5u^2 + 7u + 5)/(1+u)^3 K_{2/3}(2u/(3chi)) du
    got = _x_integral(oracle, chi, 0)
    ref = 2 / (9 * chi) * _bk_integral(chi, lambda u: 5 * u * u + 7 * u + 5, 3)
    assert got == pytest.approx(ref, rel=1e-8)


@pytest.mark.parametrize("chi", [0.05, 0.5, 2.0, 20.0])
def test_total_power_matches_baier_katkov_form(oracle, chi):
    # int x Q dx = 4/(27 chi^2) int_0^inf u (4u^2 + 5u + 4)/(1+u)^4 K_{2/3}(2u/(3chi)) du
    got = _x_integral(oracle, chi, 1)
    ref = 4 / (27 * chi * chi) * _bk_integral(chi, lambda u: u * (4 * u * u + 5 * u + 4), 4)
    assert got == pytest.approx(ref, rel=1e-8)


def test_power_small_chi_expansion(oracle):
    # radiated power over its classical value: 1 - (55 sqrt3 / 16) chi + 48 chi^2 + O(chi^3)
    # (classical int F dx = 8 pi / (9 sqrt3)).  With r(chi) = (g - 1 + c1 chi)/chi^2,
    # the Richardson combination 2 r(chi) - r(2 chi) removes the chi^3 term.
    c1 = 55 * SQ3 / 16
    classical = 8 * math.pi / (9 * SQ3)

    def r(chi):
        g = _x_integral(oracle, chi, 1) / classical
        return (g - 1 + c1 * chi) / chi ** 2

    chi = 1e-4
    r1, r2 = r(chi), r(2 * chi)
    assert abs(r1 - 48.0) < 0.1                  # the chi^2 coefficient
    assert 2 * r1 - r2 == pytest.approx(48.0, abs=0.01)


def _dn_integral_quantum(oracle, rate, chi, weight=lambda x: 1.0):
    """int_0^1 weight(x(R')) dN_q(R') dR' over both proposal branches."""
    Pa = oracle.proposal_Pa_f32()

    def f_low(v):
        r = math.exp(v)
        dn, x = oracle.trial_dn_quantum(r, rate, chi, Pa)
        return dn * weight(x) * r

    def f_up(v):
        r = -math.expm1(-v)
        dn, x = oracle.trial_dn_quantum(r, rate, chi, Pa)
        return dn * weight(x) * math.exp(-v)

    tot = 0.0
    edges = np.linspace(-240.0, math.log(Pa), 120)
    for a, b in zip(edges[:-1], edges[1:]):
        tot += integrate.quad(f_low, a, b, epsabs=0, epsrel=1e-12, limit=200)[0]
    edges = np.linspace(-math.log(1.0 - Pa), 30.0, 60)
    for a, b in zip(edges[:-1], edges[1:]):
        tot += integrate.quad(f_up, a, b, epsabs=0, epsrel=1e-12, limit=200)[0]
    return tot


def _gap(oracle, chi, g):
    """int over the x gap between the branches left by the binary32 branch point."""
    Pa = oracle.proposal_Pa_f32()
    x0 = Pa ** 0.75
    x1 = -math.log((9.0 / 7.0) * (1.0 - Pa))
    val = integrate.quad(lambda x: g(x) * oracle.quantum_kernel(x, chi)[0],
                         min(x0, x1), max(x0, x1))[0]
    return val if x1 > x0 else -val


@pytest.mark.parametrize("chi", [0.1, 1.5])
def test_quantum_estimator_is_unbiased(oracle, chi):
    # E_{R'}[dN_q] = rate int Q dx and E[eps dN_q] = rate 1.5 chi gamma int x Q dx,
    # the proposal's weights cancelling exactly (up to the branch-point gap)
    alpha, H, dt, gam = synth.ALPHA, 50.0, 0.05, 400.0
    rate = dt * SQ3 / (2 * math.pi) * alpha * H
    n_got = _dn_integral_quantum(oracle, rate, chi)
    n_ref = rate * (_x_integral(oracle, chi, 0) - _gap(oracle, chi, lambda x: 1.0))
    assert n_got == pytest.approx(n_ref, rel=1e-9)
    e_got = _dn_integral_quantum(oracle, rate, chi, weight=lambda x: 1.5 * chi * gam * x)
    e_ref = rate * 1.5 * chi * gam * (_x_integral(oracle, chi, 1) - _gap(oracle, chi, lambda x: x))
    assert e_got == pytest.approx(e_ref, rel=1e-9)


def test_quantum_step_uses_kernel_and_bounds_energy(oracle):
    """One oracle step with the quantum sampler: every trial's dN is rate Q/S at
    its x, and no photon carries more than the emitter's energy."""
    n, K = 4000, 8
    rng = np.random.default_rng(7)
    gam = 10 ** rng.uniform(2, 4.5, n)
    pm = np.sqrt(gam ** 2 - 1)
    ct = rng.uniform(-1, 1, n)
    st = np.sqrt(1 - ct ** 2)
    ph = rng.uniform(0, 2 * math.pi, n)
    state = {"px": pm * st * np.cos(ph), "py": pm * st * np.sin(ph), "pz": pm * ct,
             "w": np.ones(n), "id": np.arange(n, dtype=np.uint32), "x": None, "y": None, "z": None}
    hbar_n = 2e-4
    field = oracle.Field(0, b0=(0.0, 0.0, 300.0))
    phot, led, det = oracle.step(state, field, 0.01, 99, 3, hbar_n=hbar_n, alpha=synth.ALPHA,
                                 n_samples=K, recoil=oracle.RECOIL_NONE, kin_cut=False,
                                 sampler=oracle.SAMPLER_QUANTUM, detail=True)
    chi = np.repeat(det["chi"], K)
    assert chi.max() > 1.0                              # the regime the kernel is for
    H = np.repeat(det["heff"], K)
    rate = 0.01 * SQ3 / (2 * math.pi) * synth.ALPHA * H
    Pa = oracle.proposal_Pa_f32()
    rp, xs = det["rp"], det["xs"]
    S = np.where(rp <= Pa, (4 / 3) * rp ** 0.25, 1 - rp)
    idx = rng.choice(n * K, 400, replace=False)
    q = oracle.quantum_kernel(xs[idx], chi[idx])
    np.testing.assert_allclose(det["dn"][idx], rate[idx] * q / S[idx], rtol=1e-13, atol=0)
    gb = det["gamma_bar"][phot["parent"]]
    assert phot["eps"].size > 50
    assert (phot["eps"] < gb).all()
