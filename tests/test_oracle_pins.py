"""Pins of the FP64 oracle against what the paper and the mathematics fix.

Each test checks one part of the oracle against a value that does not come
from the oracle itself: a number printed in the paper, a closed form, an
independent library routine (scipy / mpmath / PyTorch's Philox engine), or a
brute-force quadrature.  These run on the CPU (no GPU marker).
"""
import math
import os
import shutil
import subprocess
import tempfile

import numpy as np
import pytest
from scipy import integrate, special

import synth

PI = math.pi


def _golden():
    path = os.path.join(os.path.dirname(__file__), "golden", "paper_constants.txt")
    out = {}
    for line in open(path):
        if line.strip() and not line.startswith("#"):
            name, val, tol = line.split()[:3]
            out[name] = (float(val), float(tol))
    return out


# ------------------------------------------------------------------ proposal S(x)
def test_proposal_constant_matches_paper(oracle):
    # Section "Monte Carlo method": a ~ 0.69021 makes int S = 1.
    a = oracle.proposal_a()
    val, tol = _golden()["proposal_a"]
    assert abs(a - val) < tol
    # normalisation from the closed-form integrals of the two pieces
    lower = a ** (4.0 / 3.0)                 # int_0^a (4/3) x^{1/3} dx
    upper = (7.0 / 9.0) * math.exp(-a)       # int_a^inf (7/9) e^{-x} dx
    assert abs(lower + upper - 1.0) < 1e-15
    # Pa is binary32-exact
    Pa = oracle.proposal_Pa_f32()
    assert float(np.float32(Pa)) == Pa
    assert abs(Pa - lower) < 6e-8


def test_proposal_inverse_mean_closed_form(oracle):
    # int_0^1 x(R') dR' = E_S[x] = (4/7) a^{7/3} + (7/9)(a+1) e^{-a}
    a = oracle.proposal_a()
    Pa = oracle.proposal_Pa_f32()
    expect = (4.0 / 7.0) * a ** (7.0 / 3.0) + (7.0 / 9.0) * (a + 1.0) * math.exp(-a)
    f = lambda r: oracle.proposal_invert(r, Pa)[0]
    m1, _ = integrate.quad(f, 0.0, Pa, epsabs=1e-14, epsrel=1e-13, limit=200)
    # upper branch: substitute v = -ln(1-R') to tame the log singularity
    g = lambda v: oracle.proposal_invert(-math.expm1(-v), Pa)[0] * math.exp(-v)
    m2, _ = integrate.quad(g, -math.log(1.0 - Pa), 36.0, epsabs=1e-14, epsrel=1e-13, limit=200)
    # Pa is the binary32 rounding of a^{4/3}: the branch point moves by < 3e-8
    assert abs((m1 + m2) - expect) < 1e-7


def test_proposal_density_is_derivative_of_cdf(oracle):
    # dx/dR' = 1/S(x): the returned S must be the density of the returned x
    Pa = oracle.proposal_Pa_f32()
    for r in [1e-6, 1e-3, 0.1, 0.3, 0.55, 0.65, 0.8, 0.95, 0.999]:
        h = 1e-7 * min(r, 1 - r)
        xp, _ = oracle.proposal_invert(r + h, Pa)
        xm, _ = oracle.proposal_invert(r - h, Pa)
        _, S = oracle.proposal_invert(r, Pa)
        assert abs((xp - xm) / (2 * h) * S - 1.0) < 1e-6, r


# ------------------------------------------------------------------ synchrotron F
def _F_scipy(x):
    val, _ = integrate.quad(lambda t: special.kv(5.0 / 3.0, t), x, np.inf, epsabs=0, epsrel=1e-13,
                            limit=500)
    return x * val


@pytest.mark.parametrize("x", [1e-3, 3e-3, 0.01, 0.05, 0.1, 0.2858, 0.5, 1.0, 2.0, 5.0, 10.0])
def test_F_matches_scipy_bessel_quadrature(oracle, x):
    assert oracle.synchrotron_F(x)[0] == pytest.approx(_F_scipy(x), rel=2e-10)


@pytest.mark.parametrize("x", [3.8e-6, 1e-4, 0.7, 16.4])
def test_F_matches_mpmath(oracle, x):
    mpmath = pytest.importorskip("mpmath")
    mpmath.mp.dps = 30
    ref = x * mpmath.quad(lambda t: mpmath.besselk(mpmath.mpf(5) / 3, t), [x, x + 1, mpmath.inf])
    assert oracle.synchrotron_F(x)[0] == pytest.approx(float(ref), rel=1e-12)


def test_F_quadrature_converged(oracle):
    xs = np.geomspace(3e-6, 20.0, 60)
    a = oracle.synchrotron_F(xs, 0.1)
    b = oracle.synchrotron_F(xs, 0.05)
    assert np.max(np.abs(a / b - 1.0)) < 1e-14


def test_F_small_x_asymptote(oracle):
    # F(x) = (4 pi / (sqrt3 Gamma(1/3))) (x/2)^{1/3} [1 - (Gamma(1/3)/2)(x/2)^{2/3} + O(x^2)]
    c = 4 * PI / (math.sqrt(3) * special.gamma(1 / 3))
    for x in [1e-10, 1e-8]:
        approx = c * (x / 2) ** (1 / 3) * (1 - special.gamma(1 / 3) / 2 * (x / 2) ** (2 / 3))
        assert oracle.synchrotron_F(x)[0] == pytest.approx(approx, rel=1e-9)


def test_F_large_x_asymptote(oracle):
    # F(x) ~ sqrt(pi x / 2) e^{-x} (1 + 55/(72 x) + ...)
    x = 200.0
    approx = math.sqrt(PI * x / 2) * math.exp(-x) * (1 + 55 / (72 * x))
    assert oracle.synchrotron_F(x)[0] == pytest.approx(approx, rel=5e-5)


def _quad_log(f, a, b):
    """int_a^b f(x) dx with the substitution x = e^u, split into decades."""
    edges = np.geomspace(a, b, 40)
    tot = 0.0
    for lo, hi in zip(edges[:-1], edges[1:]):
        v, _ = integrate.quad(lambda u: f(math.exp(u)) * math.exp(u), math.log(lo), math.log(hi),
                              epsabs=0, epsrel=1e-13, limit=200)
        tot += v
    return tot


def _small_x_number_tail(lo):
    """int_0^lo F(x)/x dx from the leading small-x term of F (relative error ~lo^{2/3})."""
    c = 4 * PI / (math.sqrt(3) * special.gamma(1 / 3)) / 2 ** (1 / 3)
    return 3 * c * lo ** (1 / 3)


def test_F_integral_normalisation(oracle):
    # Eq. SynchrotronFunction: (9 sqrt3 / 8 pi) F integrates to 1 over x
    F = lambda x: oracle.synchrotron_F(x)[0]
    tot = _quad_log(F, 1e-14, 60.0)
    val, tol = _golden()["bracket_integral"]
    assert tot * 9 * math.sqrt(3) / (8 * PI) == pytest.approx(val, abs=tol)


@pytest.mark.parametrize("mu", [-1, 1, 2])
def test_F_moments_closed_form(oracle, mu):
    # int x^mu F dx = 2^{mu+1}/(mu+2) Gamma(mu/2 + 7/3) Gamma(mu/2 + 2/3)
    expect = 2 ** (mu + 1) / (mu + 2) * special.gamma(mu / 2 + 7 / 3) * special.gamma(mu / 2 + 2 / 3)
    if mu == -1:
        assert expect == pytest.approx(5 * PI / 3, rel=1e-14)
    F = lambda x: oracle.synchrotron_F(x)[0] * x ** mu
    lo = 1e-14 if mu >= 0 else 1e-45
    tail = _small_x_number_tail(lo) if mu == -1 else 0.0
    assert _quad_log(F, lo, 80.0) + tail == pytest.approx(expect, rel=1e-10)


@pytest.mark.parametrize("x", [1e-5, 1e-2, 0.3, 1.0, 4.0, 15.0])
def test_number_and_energy_integrals(oracle, x):
    F = lambda t: oracle.synchrotron_F(t)[0]
    n_ref = _quad_log(lambda t: F(t) / t, 1e-30, x) + _small_x_number_tail(1e-30)
    e_ref = _quad_log(F, 1e-30, x)
    assert oracle.number_integral(x) == pytest.approx(n_ref, rel=1e-10)
    assert oracle.energy_integral(x) == pytest.approx(e_ref, rel=1e-10)
    assert oracle.number_integral(math.inf) == pytest.approx(5 * PI / 3, rel=1e-14)
    assert oracle.energy_integral(math.inf) == pytest.approx(8 * PI / (9 * math.sqrt(3)), rel=1e-14)


@pytest.mark.parametrize("chi,cut", [(1e-3, False), (0.3, True), (2.0, True)])
def test_inverse_number_cdf(oracle, chi, cut):
    xmax = 2 / (3 * chi) if cut else math.inf
    total = oracle.number_integral(xmax)
    for u in [1e-6, 0.01, 0.3, 0.5, 0.9, 0.999]:
        x = oracle.inv_number_cdf(chi, u, cut)
        assert oracle.number_integral(x) / total == pytest.approx(u, rel=1e-12)
        assert x <= xmax


# ------------------------------------------------------------------ dN estimator
def _dn_integral(oracle, rate, xcut, weight=lambda x: 1.0):
    """int_0^1 weight(x(R')) dN(R') dR' by quadrature over both branches."""
    Pa = oracle.proposal_Pa_f32()

    def f_low(v):          # R' = e^v on (0, Pa]
        r = math.exp(v)
        dn, x = oracle.trial_dn(r, rate, xcut, Pa)
        return dn * weight(x) * r

    def f_up(v):           # R' = 1 - e^{-v} on (Pa, 1)
        r = -math.expm1(-v)
        dn, x = oracle.trial_dn(r, rate, xcut, Pa)
        return dn * weight(x) * math.exp(-v)

    tot = 0.0
    edges = np.linspace(-240.0, math.log(Pa), 120)
    for a, b in zip(edges[:-1], edges[1:]):
        tot += integrate.quad(f_low, a, b, epsabs=0, epsrel=1e-12, limit=200)[0]
    edges = np.linspace(-math.log(1.0 - Pa), 30.0, 60)
    for a, b in zip(edges[:-1], edges[1:]):
        tot += integrate.quad(f_up, a, b, epsabs=0, epsrel=1e-12, limit=200)[0]
    return tot


def _branch_gap(oracle, g):
    """int over the x gap left between the two branches by the binary32 branch
    point Pa (lower branch ends at Pa^{3/4}, upper starts at -ln(9/7 (1-Pa)))."""
    Pa = oracle.proposal_Pa_f32()
    x0 = Pa ** 0.75
    x1 = -math.log((9.0 / 7.0) * (1.0 - Pa))
    return integrate.quad(lambda x: g(x) * oracle.synchrotron_F(x)[0], min(x0, x1), max(x0, x1))[0] \
        * (1.0 if x1 > x0 else -1.0)


def test_expected_photon_number_equals_rate(oracle):
    # E_{R'}[dN] = dt (sqrt3/2pi) alpha H int F/x = (5/(2 sqrt3)) alpha H dt
    alpha, H, dt = synth.ALPHA, 3.0, 0.05
    rate = dt * math.sqrt(3) / (2 * PI) * alpha * H
    got = _dn_integral(oracle, rate, math.inf)
    gap = rate * _branch_gap(oracle, lambda x: 1.0 / x)
    assert abs(gap) < 5e-8 * rate
    assert got == pytest.approx(5 / (2 * math.sqrt(3)) * alpha * H * dt - gap, rel=1e-11)


def test_expected_emitted_energy_equals_synchrotron_power(oracle):
    # E_{R'}[eps dN] with eps = 1.5 chi gamma x equals (2/3) alpha hbar_n H^2 gamma^2 dt
    alpha, hbar_n, H, gam, dt = synth.ALPHA, 3e-6, 700.0, 300.0, 0.05
    chi = hbar_n * H * gam
    rate = dt * math.sqrt(3) / (2 * PI) * alpha * H
    got = _dn_integral(oracle, rate, math.inf, weight=lambda x: 1.5 * chi * gam * x)
    gap = rate * 1.5 * chi * gam * _branch_gap(oracle, lambda x: 1.0)
    expect = (2 / 3) * alpha * hbar_n * H * H * gam * gam * dt
    assert got == pytest.approx(expect - gap, rel=1e-11)


def test_expected_number_with_kinematic_cut(oracle):
    alpha, H, dt, chi = synth.ALPHA, 100.0, 0.05, 0.8
    rate = dt * math.sqrt(3) / (2 * PI) * alpha * H
    xcut = 2 / (3 * chi)
    got = _dn_integral(oracle, rate, xcut)
    gap = rate * _branch_gap(oracle, lambda x: 1.0 / x)
    assert got == pytest.approx(rate * oracle.number_integral(xcut) - gap, rel=1e-11)


# ------------------------------------------------------------------ Philox
def _aten_philox_binary(tmpdir):
    torch = pytest.importorskip("torch")
    inc = os.path.join(os.path.dirname(torch.__file__), "include")
    if not os.path.exists(os.path.join(inc, "ATen", "core", "PhiloxRNGEngine.h")):
        pytest.skip("ATen Philox header not available")
    if shutil.which("g++") is None:
        pytest.skip("g++ not available")
    src = os.path.join(os.path.dirname(__file__), "philox_aten_ref.cpp")
    exe = os.path.join(tmpdir, "philox_ref")
    subprocess.run(["g++", "-O1", "-std=c++17", "-I" + inc, "-o", exe, src], check=True)
    return exe


def test_philox_matches_aten_engine(oracle):
    rng = np.random.default_rng(1234)
    ctr = rng.integers(0, 2 ** 32, size=(500, 4), dtype=np.uint64).astype(np.uint32)
    ctr[0] = 0
    ctr[1] = 0xFFFFFFFF
    with tempfile.TemporaryDirectory() as d:
        exe = _aten_philox_binary(d)
        keys = [np.array([0, 0], np.uint32), np.array([0xFFFFFFFF, 0xFFFFFFFF], np.uint32),
                rng.integers(0, 2 ** 32, size=2, dtype=np.uint64).astype(np.uint32)]
        for key in keys:
            text = "\n".join(" ".join(str(int(v)) for v in list(c) + list(key)) for c in ctr)
            out = subprocess.run([exe], input=text, capture_output=True, text=True, check=True).stdout
            ref = np.array([[int(t) for t in line.split()] for line in out.strip().splitlines()],
                           dtype=np.uint64).astype(np.uint32)
            got = oracle.philox4x32_10(ctr, key)
            assert np.array_equal(got, ref)


# ------------------------------------------------------------------ Boris and H_eff
def test_boris_pure_magnetic_rotation(oracle):
    # |p| is conserved and the rotation angle is 2 atan(|B| dt / (2 gamma))
    rng = np.random.default_rng(7)
    for _ in range(20):
        p = rng.normal(0, 50, 3)
        B = rng.normal(0, 3, 3)
        dt = 0.05
        pn = oracle.boris(p, [0, 0, 0], B, -1.0, dt)
        assert np.linalg.norm(pn) == pytest.approx(np.linalg.norm(p), rel=1e-14)
        bh = B / np.linalg.norm(B)
        pp, qp = p - bh * p.dot(bh), pn - bh * pn.dot(bh)
        ang = math.acos(np.clip(pp.dot(qp) / (np.linalg.norm(pp) * np.linalg.norm(qp)), -1, 1))
        g = math.sqrt(1 + p.dot(p))
        assert ang == pytest.approx(2 * math.atan(np.linalg.norm(B) * dt / (2 * g)), rel=1e-9)
        # electron (q = -1) rotates anticlockwise about B: (p x p_new) . B > 0
        assert np.cross(pp, qp).dot(B) > 0


def test_boris_pure_electric_kick(oracle):
    p = np.array([0.3, -2.0, 5.0])
    E = np.array([10.0, -4.0, 1.0])
    pn = oracle.boris(p, E, [0, 0, 0], -1.0, 0.1)
    assert np.allclose(pn, p - 0.1 * E, rtol=0, atol=1e-14)


@pytest.mark.parametrize("gamma", [1.5, 10.0, 1e3, 1e4])
@pytest.mark.parametrize("pitch", [90.0, 60.0, 10.0])
def test_heff_closed_form_uniform_B(oracle, gamma, pitch):
    # After a Boris step in a pure field B the momenta differ by a rotation of
    # angle phi with tan(phi/2) = B dt/(2 gamma); the dp_perp/p ratio is then
    # 2 p_perp sin(phi/2) / sqrt(p_perp^2 cos^2(phi/2) + p_par^2).
    Bmag, dt = 1.0, 0.02 * PI
    th = math.radians(pitch)
    pm = math.sqrt(gamma * gamma - 1)
    p = np.array([pm * math.sin(th), 0.0, pm * math.cos(th)])
    pn = oracle.boris(p, [0, 0, 0], [0, 0, Bmag], -1.0, dt)
    H, gb, r = oracle.heff(p, pn, dt)
    half = math.atan(Bmag * dt / (2 * gamma))
    pperp, ppar = pm * math.sin(th), pm * math.cos(th)
    ratio = 2 * pperp * math.sin(half) / math.sqrt((pperp * math.cos(half)) ** 2 + ppar ** 2)
    assert gb == pytest.approx(gamma, rel=1e-14)
    assert r == pytest.approx(ratio, rel=1e-9)
    assert H == pytest.approx(gamma * ratio / dt, rel=1e-9)
    if pitch == 90.0:
        # H_eff = |B| for p perpendicular to B (section "Numerical implementation")
        assert H == pytest.approx(Bmag, rel=1e-12)
    elif gamma >= 10.0:
        # small rotation per step: H_eff -> B sin(pitch)
        assert H == pytest.approx(Bmag * math.sin(th), rel=1e-4)


def test_heff_limiter_back_turn(oracle):
    # E nearly stops the particle in the first half kick, B turns it around, the
    # second half kick accelerates it backwards: dp_perp/p > 1 is capped at 1.
    dt = 0.1
    p = np.array([1.0, 0.05, 0.0])
    E = np.array([2.0 * 0.999 / dt, 0.0, 0.0])   # q = -1: half kick -dt/2 E
    B = np.array([0.0, 0.0, 400.0])
    pn = oracle.boris(p, E, B, -1.0, dt)
    H, gb, r = oracle.heff(p, pn, dt)
    assert r > 1.0
    assert H == gb / dt


def test_heff_zero_momentum(oracle):
    H, gb, r = oracle.heff([0, 0, 0], [0, 0, 0], 0.1)
    assert H == 0.0 and gb == 1.0


# ------------------------------------------------------------------ gather
def _linear_grid(n, dim):
    nx, ny, nz = n
    if dim == 2:
        nz = 1
    k, j, i = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    comps = []
    offs = synth.yee_offsets()
    coef = [(1, 2, 3), (4, -1, 2), (-3, 5, 1), (2, 2, -2), (1, -4, 3), (-1, 1, 5)]
    for c in range(6):
        cx, cy, cz = coef[c]
        v = cx * (i + offs[c][0]) + cy * (j + offs[c][1]) + (cz * (k + offs[c][2]) if dim == 3 else 0)
        comps.append(v.astype(np.float32).reshape(-1))
    return comps, coef


@pytest.mark.parametrize("dim", [2, 3])
def test_gather_reproduces_linear_field(oracle, dim):
    n = (12, 10, 8)
    dx = (0.5, 0.25, 2.0)
    comps, coef = _linear_grid(n, dim)
    f = oracle.Field(dim, n=n, dx=dx, E=comps[:3], B=comps[3:])
    rng = np.random.default_rng(3)
    offs = synth.yee_offsets()
    for _ in range(50):
        # interior positions, so the periodic wrap does not enter
        cell = rng.uniform(1.0, np.array(n) - 2.0)
        pos = cell * np.array(dx)
        E, B = oracle.gather(f, pos)
        got = np.concatenate([E, B])
        for c in range(6):
            cx, cy, cz = coef[c]
            expect = cx * cell[0] + cy * cell[1] + (cz * cell[2] if dim == 3 else 0)
            assert got[c] == pytest.approx(expect, abs=1e-12)


def test_gather_periodic_wrap(oracle):
    n = (8, 6, 4)
    f_vals = []
    rng = np.random.default_rng(11)
    for c in range(6):
        f_vals.append(rng.normal(size=n[0] * n[1] * n[2]).astype(np.float32))
    f = oracle.Field(3, n=n, dx=(1.0, 1.0, 1.0), E=f_vals[:3], B=f_vals[3:])
    # Ey at x = 7.5 (between node 7 and node 0 in x, with offset 0) and y node 2.5 -> row j=2, k=0.5
    pos = np.array([7.5, 2.5, 0.0])
    E, _ = oracle.gather(f, pos)
    a = f_vals[1].reshape(n[2], n[1], n[0])
    # Ey offset (0, 1/2, 0): u = (7.5, 2.0, 0.0) -> nodes x 7 and 0 (wrap), y 2, z 0
    expect = 0.5 * a[0, 2, 7] + 0.5 * a[0, 2, 0]
    assert E[1] == pytest.approx(float(expect), abs=1e-7)


# ------------------------------------------------------------------ one step
def _uniform_state(n, gamma, pitch_deg=90.0, seed=0):
    rng = np.random.default_rng(seed)
    pm = math.sqrt(gamma * gamma - 1)
    th = math.radians(pitch_deg)
    phi = rng.uniform(0, 2 * PI, n)
    st = {"px": pm * math.sin(th) * np.cos(phi), "py": pm * math.sin(th) * np.sin(phi),
          "pz": np.full(n, pm * math.cos(th)), "w": np.ones(n),
          "id": np.arange(n, dtype=np.uint32)}
    st["x"] = np.zeros(n)
    st["y"] = np.zeros(n)
    st["z"] = np.zeros(n)
    return st


def test_step_energy_estimator_matches_LL(oracle):
    # The expected emitted energy per trial, eps * dN, averages to the
    # synchrotron power; the LL column is beta^2 times it (eq:LLformOfRRForce).
    n, gam, B, dt, hbar_n = 1 << 16, 500.0, 2.0, 0.05, 1e-5
    st = _uniform_state(n, gam)
    f = oracle.Field(0, b0=(0, 0, B))
    ph, led, det = oracle.step(st, f, dt, 99, 0, hbar_n=hbar_n, alpha=synth.ALPHA, n_samples=4,
                               recoil=oracle.RECOIL_NONE, push_position=False, detail=True)
    eps = 1.5 * np.repeat(det["chi"] * det["gamma_bar"], 4) * det["xs"]
    mean_expected = float(np.mean(eps * det["dn"])) * n  # per particle-step, summed
    psync = (2 / 3) * synth.ALPHA * hbar_n * B * B * gam * gam * dt
    # beta of the mean momentum: the rotation by phi, tan(phi/2) = B dt/(2 gamma),
    # shortens p_bar by cos(phi/2)
    half = math.atan(B * dt / (2 * gam))
    beta2 = (1 - 1 / gam ** 2) * math.cos(half) ** 2
    assert mean_expected == pytest.approx(psync * n, rel=5e-3)
    assert led[1] == pytest.approx(beta2 * psync * n, rel=1e-9)
    # ledger "emitted" is the sum of the photon energies times weights
    assert led[0] == pytest.approx(float(np.sum(ph["w"] * ph["eps"])), rel=1e-12)
    # photon energy formula and direction
    assert np.allclose(np.linalg.norm(ph["dir"], axis=1), 1.0, atol=1e-14)


def test_step_decisions_follow_threshold(oracle):
    n = 4096
    st = _uniform_state(n, 2000.0)
    f = oracle.Field(0, b0=(0, 0, 50.0))
    ph, led, det = oracle.step(st, f, 0.05, 5, 3, hbar_n=1e-6, alpha=synth.ALPHA, n_samples=2,
                               recoil=oracle.RECOIL_NONE, push_position=False, detail=True)
    dn, b, emit = det["dn"], det["bword"].astype(np.float64), det["emit"].astype(bool)
    thr = np.floor(np.minimum(dn, 1.0) * 2.0 ** 32)
    expect = np.where(dn >= 1.0, True, b < thr)
    assert np.array_equal(emit, expect)
    assert ph["eps"].size == emit.sum()


def test_step_dn_weight_policy(oracle):
    # H dt large enough that many trials have dN >= 1: weight w dN / K (WEIGHT)
    n = 2048
    st = _uniform_state(n, 50.0)
    f = oracle.Field(0, b0=(0, 0, 2e4))
    for policy in (oracle.DN_WEIGHT, oracle.DN_CLAMP):
        s2 = {k: v.copy() for k, v in st.items()}
        ph, led, det = oracle.step(s2, f, 0.05, 1, 0, hbar_n=1e-8, alpha=synth.ALPHA, n_samples=2,
                                   dn_policy=policy, recoil=oracle.RECOIL_NONE,
                                   push_position=False, detail=True)
        big = det["dn"] >= 1.0
        assert big.sum() > 100
        wk = np.full(det["dn"].size, np.nan)
        sel = det["emit"].astype(bool)
        wk[sel] = ph["w"]
        if policy == oracle.DN_WEIGHT:
            assert np.allclose(wk[big], det["dn"][big] / 2, rtol=1e-15)
        else:
            assert np.allclose(wk[big], 0.5, rtol=0)


def test_step_kinematic_cut(oracle):
    n = 4096
    st = _uniform_state(n, 3000.0)
    f = oracle.Field(0, b0=(0, 0, 200.0))
    ph, led, det = oracle.step(st, f, 0.05, 2, 0, hbar_n=2e-3, alpha=synth.ALPHA, n_samples=4,
                               kin_cut=True, recoil=oracle.RECOIL_NONE, push_position=False,
                               detail=True)
    chi = np.repeat(det["chi"], 4)
    over = det["xs"] > 2 / (3 * chi)
    assert over.sum() > 0
    assert np.all(det["dn"][over] == 0) and not det["emit"][over].any()
    # no photon carries more energy than its emitter
    assert np.all(ph["eps"] <= np.repeat(det["gamma_bar"], 4)[det["emit"].astype(bool)] * (1 + 1e-15))


def test_step_photon_recoil_and_clamp(oracle):
    n = 512
    st = _uniform_state(n, 20.0)
    f = oracle.Field(0, b0=(0, 0, 1e4))
    s0 = {k: v.copy() for k, v in st.items()}
    s_none = {k: v.copy() for k, v in st.items()}
    kw = dict(hbar_n=3e-3, alpha=synth.ALPHA, n_samples=4, push_position=False, detail=True)
    ph, led, det = oracle.step(st, f, 0.01, 8, 0, recoil=oracle.RECOIL_PHOTON, **kw)
    _, led0, _ = oracle.step(s_none, f, 0.01, 8, 0, recoil=oracle.RECOIL_NONE, **kw)
    p_after = np.stack([st["px"], st["py"], st["pz"]], 1)
    p_push = np.stack([s_none["px"], s_none["py"], s_none["pz"]], 1)
    delta = np.zeros(n)
    np.add.at(delta, ph["parent"].astype(np.int64), ph["w"] * ph["eps"] / s0["w"][0])
    pm_push = np.linalg.norm(p_push, axis=1)
    expect_pm = np.maximum(pm_push - delta, 0.0)
    assert np.allclose(np.linalg.norm(p_after, axis=1), expect_pm, rtol=1e-12, atol=1e-12)
    clamped = np.maximum(delta - pm_push, 0.0).sum()
    assert clamped > 0
    assert led[3] == pytest.approx(clamped, rel=1e-10)
    g_after = np.sqrt(1 + (p_after ** 2).sum(1))
    g_push = np.sqrt(1 + pm_push ** 2)
    assert led[2] == pytest.approx(float((g_after - g_push).sum()), rel=1e-10)
    # direction is kept
    ok = expect_pm > 0
    cosang = (p_after[ok] * p_push[ok]).sum(1) / (np.linalg.norm(p_after[ok], axis=1) * pm_push[ok])
    assert np.allclose(cosang, 1.0, atol=1e-12)
    # photons and LL do not depend on the recoil mode within the step
    assert led[1] == led0[1]


def test_step_ll_recoil(oracle):
    n = 256
    st = _uniform_state(n, 300.0)
    s_none = {k: v.copy() for k, v in st.items()}
    f = oracle.Field(0, b0=(0, 0, 300.0))
    kw = dict(hbar_n=3e-6, alpha=synth.ALPHA, n_samples=1, push_position=False, detail=True)
    _, led, det = oracle.step(st, f, 0.05, 8, 0, recoil=oracle.RECOIL_LL, **kw)
    oracle.step(s_none, f, 0.05, 8, 0, recoil=oracle.RECOIL_NONE, **kw)
    pm_after = np.sqrt(st["px"] ** 2 + st["py"] ** 2 + st["pz"] ** 2)
    pm_push = np.sqrt(s_none["px"] ** 2 + s_none["py"] ** 2 + s_none["pz"] ** 2)
    # |dp| = dt |f_RR| = dt (2/3)(alpha/hbar_n) chi^2 beta
    chi, gb = det["chi"], det["gamma_bar"]
    # p perpendicular to B: |p| is conserved by the push, |p_bar| = |p| cos(phi/2)
    half = math.atan(300.0 * 0.05 / (2 * gb[0]))
    pbar = np.sqrt(gb ** 2 - 1) * math.cos(half)
    expect = 0.05 * (2 / 3) * (synth.ALPHA / 3e-6) * chi ** 2 * pbar / gb
    assert np.allclose(pm_push - pm_after, expect, rtol=1e-8)
    # energy lost matches the LL ledger to O(beta^2 dt-corrections)
    assert -led[2] == pytest.approx(led[1], rel=1e-2)


def test_step_position_push_periodic(oracle):
    cfg = synth.config("c2", n_particles=64, grid=(16, 16, 1))
    E, B = synth.standing_wave_grid(cfg, 0.0)
    st = {k: v.astype(np.float64) if v.dtype != np.uint32 else v
          for k, v in synth.gen_particles(cfg).items()}
    st["px"][:] = 50.0
    st["x"][:] = cfg.box[0] - 1e-3
    f = oracle.Field(2, n=cfg.grid, dx=(cfg.dx,) * 3, E=E, B=B)
    oracle.step(st, f, cfg.dt, 1, 0, hbar_n=cfg.hbar_n, alpha=cfg.alpha)
    assert np.all(st["x"] >= 0) and np.all(st["x"] < cfg.box[0])
    assert np.all(st["x"] < 1.0)  # wrapped to the start of the box


def test_step_is_order_independent(oracle):
    cfg = synth.config("c2", n_particles=2000, grid=(64, 64, 1))
    E, B = synth.standing_wave_grid(cfg, 0.3)
    base = {k: v.astype(np.float64) if v.dtype != np.uint32 else v.copy()
            for k, v in synth.gen_particles(cfg).items()}
    base["px"] *= 3000.0
    f = oracle.Field(2, n=cfg.grid, dx=(cfg.dx,) * 3, E=E, B=B)
    s1 = {k: v.copy() for k, v in base.items()}
    perm = np.random.default_rng(0).permutation(2000)
    s2 = {k: v[perm].copy() for k, v in base.items()}
    kw = dict(hbar_n=cfg.hbar_n, alpha=cfg.alpha, n_samples=2)
    ph1, led1, _ = oracle.step(s1, f, cfg.dt, 42, 7, **kw)
    ph2, led2, _ = oracle.step(s2, f, cfg.dt, 42, 7, **kw)
    inv = np.argsort(perm)
    for k in ("x", "y", "px", "py", "pz"):
        assert np.array_equal(s1[k], s2[k][inv])
    o1 = np.lexsort((ph1["k"], ph1["parent"]))
    o2 = np.lexsort((ph2["k"], ph2["parent"]))
    assert ph1["eps"].size > 0
    assert np.array_equal(ph1["eps"][o1], ph2["eps"][o2])
    assert np.allclose(led1, led2, rtol=1e-13)


def test_step_nonfinite_field_value_is_contained(oracle):
    # A NaN grid value reaches only the particles whose cloud-in-cell stencil
    # holds that node (found here geometrically): they come out non-finite,
    # emit nothing and add nothing to the ledger; every other particle, its
    # photons and the ledger are those of the same step without the NaN.
    cfg = synth.config("c3", grid=(12, 10, 8), slab=None)
    E, B = synth.standing_wave_grid(cfg, 0.4)
    base = {k: v.astype(np.float64) if v.dtype != np.uint32 else v.copy()
            for k, v in synth.gen_particles(cfg, n=3000).items()}
    for k in ("px", "py", "pz"):
        base[k] *= 3000.0
    node = (5, 4, 3)                 # Ex node (i + 1/2, j, k)
    nx, ny, nz = cfg.grid
    j_flat = node[0] + nx * (node[1] + ny * node[2])
    E_bad = [a.copy() for a in E]
    E_bad[0][j_flat] = np.float32(np.nan)
    kw = dict(hbar_n=cfg.hbar_n, alpha=cfg.alpha, n_samples=4, kin_cut=True)
    f_ok = oracle.Field(3, n=cfg.grid, dx=(cfg.dx,) * 3, E=E, B=B)
    f_bad = oracle.Field(3, n=cfg.grid, dx=(cfg.dx,) * 3, E=E_bad, B=B)
    # stencil of Ex: base node floor(x/dx - 1/2), floor(y/dx), floor(z/dx) and +1, periodic
    u = np.stack([base["x"] / cfg.dx - 0.5, base["y"] / cfg.dx, base["z"] / cfg.dx], 1)
    i0 = np.floor(u).astype(np.int64)
    hit = np.ones(3000, bool)
    for a, (nn, c) in enumerate(zip(cfg.grid, node)):
        hit &= (((i0[:, a] - c) % nn) == 0) | (((i0[:, a] + 1 - c) % nn) == 0)
    assert 0 < hit.sum() < 100
    s_ok = {k: v.copy() for k, v in base.items()}
    s_bad = {k: v.copy() for k, v in base.items()}
    s_sub = {k: v[~hit].copy() for k, v in base.items()}
    ph_ok, led_ok, _ = oracle.step(s_ok, f_ok, cfg.dt, 5, 2, **kw)
    ph_bad, led_bad, det = oracle.step(s_bad, f_bad, cfg.dt, 5, 2, detail=True, **kw)
    _, led_sub, _ = oracle.step(s_sub, f_ok, cfg.dt, 5, 2, **kw)
    p_bad = np.stack([s_bad[k] for k in ("px", "py", "pz")], 1)
    assert np.array_equal(~np.isfinite(p_bad).all(1), hit)
    assert np.all(det["heff"][hit] == 0) and np.all(det["chi"][hit] == 0)
    for k in ("x", "y", "z", "px", "py", "pz"):
        assert np.array_equal(s_bad[k][~hit], s_ok[k][~hit])
    assert not np.isin(ph_bad["parent"], base["id"][hit]).any()
    keep = ~np.isin(ph_ok["parent"], base["id"][hit])
    assert ph_bad["eps"].size == keep.sum() > 0
    assert np.array_equal(ph_bad["eps"], ph_ok["eps"][keep])
    assert np.all(np.isfinite(led_bad))
    np.testing.assert_allclose(led_bad, led_sub, rtol=1e-12, atol=0)
