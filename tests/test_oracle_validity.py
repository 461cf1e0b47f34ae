"""Pins of the oracle's grid-frequency floor (section "The field setup": the
grid resolves radiation below omega_grid = c/dx, so only photons above it are
emitted as particles).

The floor must change nothing but the emission of photons below hbar
omega_grid: with the same random numbers the photons with it are exactly the
photons without it whose energy is at least hbar omega_grid, and the momenta
differ only where a recoil came from a removed photon."""
import numpy as np
import pytest

import synth


def _state(cfg, n):
    st = synth.gen_particles(cfg, n=n)
    return {k: (v.astype(np.float64) if v.dtype != np.uint32 else v.copy()) for k, v in st.items()}


@pytest.mark.parametrize("sampler", [0, 1, 2])
def test_floor_removes_exactly_the_photons_below_it(oracle, sampler):
    cfg = synth.config("c1", b0=(0.0, 0.0, 40.0), gamma_range=(1e2, 1e4))
    n, K = 3000, 4
    field = oracle.Field(0, b0=cfg.b0)
    kw = dict(hbar_n=cfg.hbar_n, alpha=cfg.alpha, n_samples=K, recoil=oracle.RECOIL_PHOTON,
              kin_cut=sampler == 1, sampler=sampler, push_position=False, detail=True)
    s0 = _state(cfg, n)
    s1 = _state(cfg, n)
    for s in (s0, s1):
        s["x"] = s["y"] = s["z"] = None
    ph0, led0, det0 = oracle.step(s0, field, cfg.dt, 5, 2, **kw)
    # a grid frequency inside the emitted band: about half the photons are below it
    e_med = float(np.median(ph0["eps"]))
    omega_grid = e_med / cfg.hbar_n
    ph1, led1, det1 = oracle.step(s1, field, cfg.dt, 5, 2, omega_grid=omega_grid, **kw)
    keep = ph0["eps"] >= cfg.hbar_n * omega_grid
    assert 0.2 < keep.mean() < 0.8
    for k in ("eps", "w", "parent", "k"):
        assert np.array_equal(ph1[k], ph0[k][keep]), k
    # decisions before the floor, dN and the push are untouched
    assert np.array_equal(det1["dn"], det0["dn"])
    assert np.array_equal(det1["heff"], det0["heff"])
    # the emitted-energy column is the kept photons' energy; LL is unchanged
    assert led1[0] == pytest.approx(float(np.sum(ph0["w"][keep] * ph0["eps"][keep])), rel=1e-12)
    assert led1[1] == led0[1]
    # momenta change only for particles that lost a photon
    lost = np.unique(ph0["parent"][~keep])
    same = np.ones(n, bool)
    same[lost] = False
    for k in ("px", "py", "pz"):
        assert np.array_equal(s1[k][same], s0[k][same])
    assert not np.array_equal(s1["px"][lost], s0["px"][lost])


def test_floor_zero_is_no_floor(oracle):
    cfg = synth.config("c1", b0=(0.0, 0.0, 40.0))
    field = oracle.Field(0, b0=cfg.b0)
    out = []
    for og in (0.0, None):
        s = _state(cfg, 2000)
        s["x"] = s["y"] = s["z"] = None
        kw = dict(hbar_n=cfg.hbar_n, alpha=cfg.alpha, n_samples=2, push_position=False)
        if og is not None:
            kw["omega_grid"] = og
        out.append(oracle.step(s, field, cfg.dt, 9, 1, **kw)[0])
    assert np.array_equal(out[0]["eps"], out[1]["eps"])


def test_validity_flags_closed_form(oracle):
    # uniform B, pure magnetic rotation: H_eff = B sin(pitch) (to the push's
    # O(dt^2) turning correction) and chi = hbar_n H_eff gamma, so the flags
    # follow from gamma, pitch and B alone
    B, hbar_n, tau_em, dt = 40.0, 1e-4, 0.03, 1e-3
    n = 4000
    rng = np.random.default_rng(3)
    gam = 10.0 ** rng.uniform(0.5, 3.5, n)
    ct = rng.uniform(-1, 1, n)
    pm = np.sqrt(gam ** 2 - 1)
    st = np.sqrt(1 - ct ** 2)
    s = {"px": pm * st, "py": np.zeros(n), "pz": pm * ct, "w": np.ones(n),
         "id": np.arange(n, dtype=np.uint32), "x": None, "y": None, "z": None}
    _, _, det = oracle.step(s, oracle.Field(0, b0=(0.0, 0.0, B)), dt, 1, 0, hbar_n=hbar_n,
                            alpha=synth.ALPHA, push_position=False, recoil=0, detail=True)
    # pitch angle to B = z: sin = st
    h = B * st
    c = hbar_n * h * gam
    f = oracle.validity_flags(det["heff"], det["chi"], tau_em)
    away = (np.abs(c - 1) > 1e-3) & (np.abs(h * tau_em - 1) > 1e-3)
    expect = np.where(c >= 1, 1, 0) | np.where((h > 0) & (h * tau_em <= 1), 2, 0)
    assert np.array_equal(f[away], expect[away])
    assert (f & 1).any() and (f & 2).any() and (f == 0).any()
