"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle on the
same seeded inputs.  Tolerances are defined in tests/parity.py."""
from __future__ import annotations

import math
import sys

import numpy as np
import pytest

import synth
from tests import parity

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _say(msg):
    print(f"[gpu-case] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def sr():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1409_5574_amd import api
    api.lib()
    return api


@pytest.fixture(scope="module")
def table(sr):
    _say("table build")
    t = sr.Table()
    torch.cuda.synchronize()
    return t


# ------------------------------------------------------------------ primitives
def test_philox_bit_exact(sr, oracle):
    rng = np.random.default_rng(5)
    ctr = rng.integers(0, 2 ** 32, size=(4096, 4), dtype=np.uint64).astype(np.uint32)
    seed = 0x0123456789ABCDEF
    _say("philox 4096")
    got = sr.philox(torch.from_numpy(ctr.view(np.int32)), seed).cpu().numpy().view(np.uint32)
    ref = oracle.philox4x32_10(ctr, [seed & 0xFFFFFFFF, seed >> 32])
    assert np.array_equal(got, ref)


def test_table_constants(sr, table, oracle):
    info = table.info()
    assert info.proposal_pa == np.float32(oracle.proposal_Pa_f32())
    assert info.proposal_a == pytest.approx(oracle.proposal_a(), rel=1e-15)


def test_table_F_against_oracle(sr, table, oracle):
    x = np.geomspace(2.0 ** -18.4, 22.0, 20001)
    _say("eval F 20001")
    got = sr.eval_F(table, torch.from_numpy(x.astype(np.float32))).cpu().numpy().astype(np.float64)
    ref = oracle.synchrotron_F(x.astype(np.float32).astype(np.float64))
    rel = np.abs(got / ref - 1.0)
    assert rel.max() < 3e-6, rel.max()


def test_trial_dn_against_oracle(sr, table, oracle):
    rng = np.random.default_rng(9)
    n = 20000
    a = rng.integers(0, 2 ** 32, size=n, dtype=np.uint64).astype(np.uint32)
    rate = np.float32(0.013)
    chi = np.full(n, 0.4, np.float32)
    _say("eval trial 20000")
    dn, xg = sr.eval_trial(table, torch.from_numpy(a.view(np.int32)),
                           torch.full((n,), float(rate)), torch.from_numpy(chi), False)
    dn, xg = dn.cpu().numpy(), xg.cpu().numpy()
    Pa = oracle.proposal_Pa_f32()
    rp = ((a >> 9).astype(np.float64) + 0.5) / 2 ** 23
    ref = np.array([oracle.trial_dn(r, float(rate), math.inf, Pa) for r in rp])
    assert np.max(np.abs(xg / ref[:, 1] - 1)) < 3e-7
    assert np.max(np.abs(dn / ref[:, 0] - 1)) < 3e-6


def test_quantum_trial_against_oracle(sr, table, oracle):
    rng = np.random.default_rng(11)
    n = 20000
    a = rng.integers(0, 2 ** 32, size=n, dtype=np.uint64).astype(np.uint32)
    chi = (10.0 ** rng.uniform(-3.0, 0.8, n)).astype(np.float32)
    rate = np.float32(0.013)
    _say("eval quantum trial 20000")
    dn, xg = sr.eval_trial_quantum(table, torch.from_numpy(a.view(np.int32)),
                                   torch.full((n,), float(rate)), torch.from_numpy(chi))
    dn = dn.cpu().numpy().astype(np.float64)
    xg = xg.cpu().numpy().astype(np.float64)
    Pa = oracle.proposal_Pa_f32()
    rp = ((a >> 9).astype(np.float64) + 0.5) / 2 ** 23
    c64 = chi.astype(np.float64)
    ref = np.array([oracle.trial_dn_quantum(r, float(rate), c, Pa) for r, c in zip(rp, c64)])
    assert np.max(np.abs(xg / ref[:, 1] - 1)) < 3e-7
    d = 1.5 * c64 * ref[:, 1]
    xi = ref[:, 1] / np.maximum(1.0 - d, 1e-300)
    # (dN below 1e-30 is under FP32's normal range once multiplied out, and far
    # below any decision: a trial emits only if dN 2^32 >= 1)
    live = (d < 1.0 - 1e-5) & (xi < 100.0) & (ref[:, 0] > 1e-30)
    dead = d >= 1.0 + 1e-5
    assert live.sum() > n // 2 and dead.sum() > 100
    # beyond the kinematic edge: exactly zero on both sides
    assert (dn[dead] == 0).all() and (ref[dead, 0] == 0).all()
    tol = parity.quantum_dn_tol(c64, ref[:, 1])
    rel = np.abs(dn[live] / ref[live, 0] - 1)
    assert (rel <= tol[live]).all(), (rel.max(), np.argmax(rel / tol[live]))
    # the bulk (away from the edge) as accurate as the classical trial table
    bulk = live & (d < 0.5) & (xi < 20.0)
    assert np.max(np.abs(dn[bulk] / ref[bulk, 0] - 1)) < 5e-6


# ------------------------------------------------------------------ one-step parity
def _orc_state(d):
    return {k: (v.astype(np.float64) if v.dtype != np.uint32 else v.copy()) for k, v in d.items()}


def run_step_case(sr, table, oracle, cfg, n, *, K=None, recoil=None, kin_cut=None, dtype=np.float32,
                  p_scale=1.0, seed=777, step=3, t=0.4, sampler=0, chunks=None, dn_policy=0,
                  label="", omega_grid=0.0, edit_state=None, edit_fields=None, status_ok=2,
                  gather=0, sort_tile=None):
    K = cfg.n_samples if K is None else K
    recoil = cfg.recoil if recoil is None else recoil
    kin_cut = cfg.kin_cut if kin_cut is None else kin_cut
    st = synth.gen_particles(cfg, n=n)
    for k in ("px", "py", "pz"):
        st[k] = (st[k].astype(np.float64) * p_scale).astype(np.float32)
    if edit_state is not None:
        edit_state(st)
    if sort_tile is not None:
        # particles ordered by tile (x fastest), as the tile sort leaves them
        key = np.zeros(n, np.int64)
        for a in reversed(range(cfg.dim)):
            q = cfg.grid[a] // sort_tile[a]
            key = key * q + (np.floor(st["xyz"[a]] / cfg.dx).astype(np.int64) // sort_tile[a])
        order = np.argsort(key, kind="stable")
        st = {k: v[order].copy() for k, v in st.items()}
    old = _orc_state(st)
    dim = cfg.dim
    if dim == 0:
        fo = oracle.Field(0, b0=cfg.b0)
        E = B = None
        grid = sr.grid_struct(0, b0=cfg.b0)
        fields = None
    else:
        E, B = synth.standing_wave_grid(cfg, t)
        if edit_fields is not None:
            edit_fields(E, B)
        fo = oracle.Field(dim, n=cfg.grid, dx=(cfg.dx,) * 3, E=E, B=B)
        grid = sr.grid_struct(dim, n=cfg.grid, dx=(cfg.dx,) * 3)
        fields = sr.Fields(E, B)
    # oracle
    orc = _orc_state(st)
    if dim == 0:
        orc["x"] = orc["y"] = orc["z"] = None
    if dim == 2:
        orc["z"] = None
    ph_o, led_o, det = oracle.step(orc, fo, cfg.dt, seed, step, hbar_n=cfg.hbar_n, alpha=cfg.alpha,
                                   n_samples=K, recoil=recoil, kin_cut=kin_cut,
                                   sampler={0: 0, 3: 2}.get(sampler, 1), dn_policy=dn_policy,
                                   push_position=dim != 0, detail=True, omega_grid=omega_grid)
    # GPU
    tdtype = torch.float64 if dtype == np.float64 else torch.float32
    gst = {k: (v if k == "id" else v.astype(dtype)) for k, v in st.items()}
    parts = sr.Particles.from_numpy(gst, dtype=tdtype, dim=dim if dim else 0)
    if dim == 0:
        parts.x = [None, None, None]
    start = None
    n_chunks = None
    if chunks is not None:
        start = torch.from_numpy(np.asarray(chunks, np.int64)).to("cuda")
        n_chunks = len(chunks) - 1
    photons = sr.PhotonBuffer(n, K, n_chunks=n_chunks, dim=dim if dim else 3)
    ledger = sr.LedgerBuf(4, n_chunks if n_chunks is not None else sr.n_chunks_uniform(n))
    prm = sr.params_struct(cfg.hbar_n, cfg.alpha, K, sampler, recoil, dn_policy, kin_cut, dim != 0,
                           omega_grid=omega_grid, gather=gather)
    _say(f"step {label} n={n} K={K} dim={dim} dtype={np.dtype(dtype).name}")
    sr.gather_push_emit(parts, fields, grid, cfg.dt, seed, step, prm, table, photons, ledger, 1,
                        start=start)
    torch.cuda.synchronize()
    gs = parts.to_numpy()
    ph_g = photons.gather(n, start)
    led_g = ledger.row(1)
    status = ledger.read_status()
    xcut_band = None
    if kin_cut:
        chi = np.repeat(det["chi"], K)
        xcut_band = np.abs(1.5 * chi * det["xs"] - 1.0) <= 1e-5
    if omega_grid > 0:
        # photons within FP32 rounding of hbar omega_grid may land on either side
        eps_x = 1.5 * np.repeat(det["chi"] * det["gamma_bar"], K) * det["xs"]
        band = np.abs(eps_x / (cfg.hbar_n * omega_grid) - 1.0) <= 1e-5
        xcut_band = band if xcut_band is None else (xcut_band | band)
    dn_tol = None
    if sampler == 3:
        dn_tol = parity.quantum_dn_tol(np.repeat(det["chi"], K), det["xs"])
    box = cfg.box if dim else None
    rep = parity.compare_step(gs, orc, old, ph_g, ph_o, det, K, box=box, xcut_band=xcut_band,
                              dn_tol=dn_tol)
    # ledger: remove the energy of flipped trials from the comparison budget
    flips_e = 0.0
    if rep["decision_flips"]:
        flips_e = float(np.abs(ph_o["w"] * ph_o["eps"]).max()) * rep["decision_flips"]
    parity.compare_ledger(led_g, led_o, flips_e,
                          cols=(0, 1, 3, 4) + ((2,) if recoil != 0 and abs(led_o[2]) > 0 else ()))
    assert led_g[5] == ph_g["count"]
    assert ph_g["count"] == ph_g["stored"]
    assert status & ~status_ok == 0, status
    # the clamp bit is set exactly when the oracle clamped some recoil
    assert bool(status & 2) == (led_o[3] > 0), (status, led_o[3])
    rep["ledger_gpu"] = led_g
    rep["ledger_orc"] = led_o
    rep["status"] = status
    rep["det"] = det
    rep["ph_g"] = ph_g
    # blocks whose partial ledger row marks a gather from the LDS field box
    nb = -(-(n_chunks if n_chunks is not None else sr.n_chunks_uniform(n)) // 4)
    part = ledger.partials[:nb * 10].view(nb, 10).cpu().numpy()
    rep["box_blocks"] = int((part[:, 9] == 1.0).sum())
    rep["blocks"] = nb
    return rep


def test_step_uniform_field(sr, table, oracle):
    cfg = synth.config("c1", b0=(0.0, 0.0, 40.0))
    rep = run_step_case(sr, table, oracle, cfg, 5000, label="uniform B=40")
    assert rep["photons_oracle"] > 50


def test_step_uniform_field_K8_ll(sr, table, oracle):
    cfg = synth.config("c1", b0=(0.0, 0.0, 40.0))
    rep = run_step_case(sr, table, oracle, cfg, 3001, K=8, recoil=2, label="uniform K8 LL")
    assert rep["photons_oracle"] > 100


def test_step_2d_grid(sr, table, oracle):
    cfg = synth.config("c2", grid=(96, 80, 1))
    rep = run_step_case(sr, table, oracle, cfg, 7777, p_scale=2000.0, label="2d 96x80")
    assert rep["photons_oracle"] > 500


def test_step_3d_grid_K8_cut(sr, table, oracle):
    cfg = synth.config("c3", grid=(24, 20, 16), slab=None)
    rep = run_step_case(sr, table, oracle, cfg, 4099, p_scale=3000.0, label="3d 24x20x16 K8")
    assert rep["photons_oracle"] > 1000


def test_step_3d_fp64_path(sr, table, oracle):
    # FP64 gather + push: without recoil the momenta agree with the oracle to
    # FP64 rounding; with recoil the FP32 photon energies set the error.
    cfg = synth.config("c5", grid=(16, 16, 12), n_particles=3000)
    rep = run_step_case(sr, table, oracle, cfg, 3000, dtype=np.float64, recoil=0,
                        label="3d fp64 no recoil")
    assert rep["p_rel_err"] < 1e-12
    rep = run_step_case(sr, table, oracle, cfg, 3000, dtype=np.float64, label="3d fp64 recoil")
    assert rep["p_rel_err"] < 1e-6


@pytest.mark.parametrize("dn_policy", [0, 1])
def test_step_dn_above_one(sr, table, oracle, dn_policy):
    # B = 3e4 at gamma 200..2000: many trials have dN >= 1 (policy 0 gives
    # them weight w dN/K, policy 1 the literal min(dN, 1) of the comparison
    # with R), and the turn per step is large enough for the limiter
    # dp_perp/p <= 1 of eq:effective_H to act
    cfg = synth.config("c1", b0=(0.0, 0.0, 3e4), gamma_range=(200.0, 2000.0))
    rep = run_step_case(sr, table, oracle, cfg, 2000, K=2, dn_policy=dn_policy,
                        label=f"dN>=1 policy {dn_policy}")
    det = rep["det"]
    assert rep["photons_oracle"] > 1000
    assert (det["dn"] >= 1.0).sum() > 500
    assert (det["ratio"] > 1.0).sum() > 100, "the limiter is not reached"
    w = rep["ph_g"]["w"]
    if dn_policy == 1:
        assert np.all(w == np.float32(0.5))      # every photon carries w/K
    else:
        assert (w > 0.5).sum() > 100              # dN >= 1 photons carry w dN/K


@pytest.mark.parametrize("sampler", [0, 3])
def test_step_field_box_gather(sr, table, oracle, sampler):
    # a dense 3D plasma (2 particles per cell) in tile order: most 256-particle
    # blocks fit their stencils in an LDS box; parity with the oracle as for the
    # direct gather (the same bits, checked below)
    cfg = synth.config("c3", grid=(40, 32, 24), slab=None)
    n = 2 * 40 * 32 * 24
    rep = run_step_case(sr, table, oracle, cfg, n, p_scale=3000.0, sampler=sampler,
                        kin_cut=sampler == 0, gather=1, sort_tile=(4, 4, 4),
                        label=f"3d field box sampler {sampler}")
    assert rep["box_blocks"] >= rep["blocks"] // 2, (rep["box_blocks"], rep["blocks"])
    assert rep["photons_oracle"] > 1000


def test_field_box_gather_is_bit_identical(sr, table):
    """SR_GATHER_BOX against SR_GATHER_DIRECT from the same state: particles,
    photon records and ledger row bit for bit, on a tile-sorted dense plasma
    (most blocks from the box), an unsorted one (every box too large: the
    fallback), and a grid of 8 cells along z where boxes wrap around the
    periodic boundary or would wrap onto themselves."""
    for grid, tile, label in (((48, 40, 32), (4, 4, 4), "sorted"), ((48, 40, 32), None, "unsorted"),
                              ((64, 48, 8), (4, 4, 4), "thin z")):
        cfg = synth.config("c3", grid=grid, slab=None)
        n = 2 * int(np.prod(grid))
        st = synth.gen_particles(cfg, n=n, seed=41)
        for k in ("px", "py", "pz"):
            st[k] = (st[k].astype(np.float64) * 2500.0).astype(np.float32)
        if tile is not None:
            key = np.zeros(n, np.int64)
            for a in (2, 1, 0):
                key = key * (grid[a] // tile[a]) + (np.floor(st["xyz"[a]] / cfg.dx).astype(np.int64)
                                                    // tile[a])
            o = np.argsort(key, kind="stable")
            st = {k: v[o].copy() for k, v in st.items()}
        E, B = synth.standing_wave_grid(cfg, 0.7)
        fields = sr.Fields(E, B)
        g = sr.grid_struct(3, n=grid, dx=(cfg.dx,) * 3)
        outs = []
        for gather in (0, 1):
            parts = sr.Particles.from_numpy(st, dim=3)
            photons = sr.PhotonBuffer(n, cfg.photons_per_particle, dim=3)
            ledger = sr.LedgerBuf(1, sr.n_chunks_uniform(n))
            prm = sr.params_struct(cfg.hbar_n, cfg.alpha, cfg.n_samples, recoil=cfg.recoil,
                                   kin_cut=True, gather=gather)
            _say(f"field box bit-identity {label} gather={gather} n={n}")
            sr.gather_push_emit(parts, fields, g, cfg.dt, 5, 3, prm, table, photons, ledger, 0)
            torch.cuda.synchronize()
            nb = -(-sr.n_chunks_uniform(n) // 4)
            used = int((ledger.partials[:nb * 10].view(nb, 10)[:, 9] == 1.0).sum().item())
            outs.append((parts.to_numpy(), photons.gather(n), ledger.row(0), used, nb))
        (pa, pha, la, _, _), (pb, phb, lb, used, nb) = outs
        for k in ("x", "y", "z", "px", "py", "pz"):
            assert np.array_equal(pa[k], pb[k]), (label, k)
        for k in ("eps", "w", "dir", "pos", "parent", "k"):
            assert np.array_equal(pha[k], phb[k]), (label, k)
        assert np.array_equal(la, lb), label
        print(f"field box {label}: {used}/{nb} blocks from the box, {pha['count']} photons",
              flush=True)
        if label == "sorted":
            assert used > nb // 2
        if label == "unsorted":
            assert used == 0


def test_step_zero_momentum_particles(sr, table, oracle):
    # p = 0 in a pure magnetic field: the mean momentum vanishes, so H_eff = 0
    # (no direction of motion): no photons, no LL loss, the momentum stays 0
    cfg = synth.config("c1", b0=(0.0, 0.0, 40.0))
    zero = np.arange(0, 3000, 3)

    def edit(st):
        for k in ("px", "py", "pz"):
            st[k][zero] = 0.0

    rep = run_step_case(sr, table, oracle, cfg, 3000, K=4, edit_state=edit, label="p = 0")
    det = rep["det"]
    assert np.all(det["heff"][zero] == 0.0)
    assert rep["photons_oracle"] > 50


def test_step_nonfinite_field_value(sr, table, oracle):
    # one NaN Ex value and one infinite Bz value: the particles whose stencil
    # holds them are non-finite on both sides, flagged, emit nothing and add
    # nothing to the ledger; every other particle is unaffected
    cfg = synth.config("c3", grid=(24, 20, 16), slab=None)
    nx, ny = cfg.grid[0], cfg.grid[1]

    def edit(E, B):
        E[0][7 + nx * (5 + ny * 4)] = np.float32(np.nan)
        B[2][15 + nx * (12 + ny * 9)] = np.float32(np.inf)

    rep = run_step_case(sr, table, oracle, cfg, 4099, p_scale=3000.0, edit_fields=edit,
                        status_ok=2 | 4, label="3d NaN/inf field")
    assert rep["status"] & 4
    assert 0 < rep["nonfinite"] < 200
    assert np.all(np.isfinite(rep["ledger_gpu"][:5]))
    assert rep["photons_oracle"] > 1000


def test_step_explicit_chunks(sr, table, oracle):
    cfg = synth.config("c2", grid=(64, 64, 1))
    chunks = [0, 1, 300, 300, 1000, 1257, 2000]
    run_step_case(sr, table, oracle, cfg, 2000, p_scale=2000.0, chunks=chunks, label="chunks")


def test_step_table_sampler(sr, table, oracle):
    cfg = synth.config("c1", b0=(0.0, 0.0, 40.0), gamma_range=(1e3, 1e4))
    rep = run_step_case(sr, table, oracle, cfg, 4000, K=2, sampler=1, kin_cut=True,
                        label="table sampler")
    assert rep["photons_oracle"] > 40


def test_step_quantum_sampler_3d(sr, table, oracle):
    # chi ~ 1 (the regime the quantum kernel is for): thermal momenta scaled up
    # in the a0 = 500 standing wave; the kinematic edge is built into the kernel
    cfg = synth.config("c3", grid=(24, 20, 16), slab=None)
    rep = run_step_case(sr, table, oracle, cfg, 4099, p_scale=6000.0, sampler=3, kin_cut=False,
                        label="3d quantum K8")
    assert rep["photons_oracle"] > 1000


def test_step_quantum_sampler_uniform_K1(sr, table, oracle):
    # chi = hbar_n B gamma sin(pitch) from 1e-2 to 10
    cfg = synth.config("c1", b0=(0.0, 0.0, 100.0), gamma_range=(1e2, 1e5), hbar_n=1e-6)
    rep = run_step_case(sr, table, oracle, cfg, 8000, K=1, sampler=3, kin_cut=False,
                        label="uniform quantum K1")
    assert rep["photons_oracle"] > 150


def _median_photon_omega(oracle, cfg, n, K, p_scale, sampler, kin_cut):
    """A grid frequency inside the emitted band of the case (about half the
    photons below it), from an oracle step of the same case."""
    st = synth.gen_particles(cfg, n=n)
    for k in ("px", "py", "pz"):
        st[k] = (st[k].astype(np.float64) * p_scale).astype(np.float32)
    orc = _orc_state(st)
    if cfg.dim == 0:
        fo = oracle.Field(0, b0=cfg.b0)
        orc["x"] = orc["y"] = orc["z"] = None
    else:
        E, B = synth.standing_wave_grid(cfg, 0.4)
        fo = oracle.Field(cfg.dim, n=cfg.grid, dx=(cfg.dx,) * 3, E=E, B=B)
    ph, _, _ = oracle.step(orc, fo, cfg.dt, 777, 3, hbar_n=cfg.hbar_n, alpha=cfg.alpha, n_samples=K,
                           recoil=cfg.recoil, kin_cut=kin_cut, sampler={0: 0, 3: 2}.get(sampler, 1),
                           push_position=cfg.dim != 0)
    return float(np.median(ph["eps"])) / cfg.hbar_n


@pytest.mark.parametrize("sampler", [0, 1, 3])
def test_step_grid_frequency_floor(sr, table, oracle, sampler):
    cfg = synth.config("c3", grid=(24, 20, 16), slab=None)
    kin_cut = sampler == 1
    og = _median_photon_omega(oracle, cfg, 4099, 8, 3000.0, sampler, kin_cut)
    rep = run_step_case(sr, table, oracle, cfg, 4099, p_scale=3000.0, sampler=sampler,
                        kin_cut=kin_cut, omega_grid=og, label=f"3d floor sampler {sampler}")
    assert rep["photons_oracle"] > 300


def test_validity_against_oracle(sr, table, oracle):
    cfg = synth.config("c3", grid=(24, 20, 16), slab=None)
    n = 6000
    st = synth.gen_particles(cfg, n=n)
    for k in ("px", "py", "pz"):
        st[k] = (st[k].astype(np.float64) * 4000.0).astype(np.float32)
    old = _orc_state(st)
    orc = _orc_state(st)
    E, B = synth.standing_wave_grid(cfg, 0.4)
    fo = oracle.Field(3, n=cfg.grid, dx=(cfg.dx,) * 3, E=E, B=B)
    _, _, det = oracle.step(orc, fo, cfg.dt, 1, 0, hbar_n=cfg.hbar_n, alpha=cfg.alpha, n_samples=1,
                            recoil=0, push_position=False, detail=True)
    tau_em = 0.02
    f_o = oracle.validity_flags(det["heff"], det["chi"], tau_em)
    pb = 0.5 * (np.stack([old[k] for k in ("px", "py", "pz")], 1)
                + np.stack([orc[k] for k in ("px", "py", "pz")], 1))
    beta2 = (pb * pb).sum(1) / det["gamma_bar"] ** 2
    parts = sr.Particles.from_numpy(st, dim=3)
    grid = sr.grid_struct(3, n=cfg.grid, dx=(cfg.dx,) * 3)
    fields = sr.Fields(E, B)
    _say("validity diagnostics")
    flags, sums = sr.validity(parts, fields, grid, cfg.dt, cfg.hbar_n, cfg.alpha, tau_em)
    torch.cuda.synchronize()
    f_g = flags.cpu().numpy()
    # away from the two thresholds the flags agree exactly
    away = (np.abs(det["chi"] - 1.0) > 1e-5) & (np.abs(det["heff"] * tau_em - 1.0) > 1e-5)
    assert np.array_equal(f_g[away], f_o[away])
    assert (f_o & 1).any() and (f_o & 2).any() and (f_o == 0).any()
    # the sums, with the oracle's definition over the GPU's flags (the flags are
    # compared above); the LL energy carries the FP32 chi error
    ref = oracle.validity_sums(st["w"], det["chi"], beta2, f_g, cfg.alpha, cfg.hbar_n, cfg.dt)
    np.testing.assert_allclose(sums[:3], ref[:3], rtol=1e-12)
    np.testing.assert_allclose(sums[3:], ref[3:], rtol=2e-5)
    # the particles are untouched
    assert np.array_equal(parts.to_numpy()["px"], st["px"])
