"""The MLP surrogate on the GPU: forward and gradients against the FP64
reference, training on the GPU, the spectrum judge and fallback map, and the
emission step driven by the network."""
from __future__ import annotations

import math
import sys

import numpy as np
import pytest

import synth
from oracle import mlp as omlp
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
    t = sr.Table()
    torch.cuda.synchronize()
    return t


def test_mlp_forward_matches_oracle(sr):
    flat = omlp.bf16_round(omlp.init(5))
    net = sr.Mlp(flat.astype(np.float32))
    rng = np.random.default_rng(2)
    f = rng.uniform(-1.3, 1.3, (5003, 2)).astype(np.float32)
    _say("mlp forward 5003")
    y = net.forward(torch.from_numpy(f)).cpu().numpy().astype(np.float64)
    ref = omlp.forward(flat, f.astype(np.float64))
    # activations enter the matrix cores as bfloat16 pairs (~16 bits)
    scale = np.abs(ref).max()
    assert np.abs(y - ref).max() <= 1e-3 * scale
    assert np.corrcoef(y, ref)[0, 1] > 0.9999


def test_mlp_gradients_match_oracle(sr):
    flat = omlp.bf16_round(omlp.init(6))
    net = sr.Mlp(flat.astype(np.float32))
    rng = np.random.default_rng(3)
    M = 4111
    f = rng.uniform(-1.2, 1.2, (M, 2)).astype(np.float32)
    t = rng.normal(-2.0, 1.5, M).astype(np.float32)
    _say("mlp grads 4111")
    g = net.mse_grad(torch.from_numpy(f).cuda(), torch.from_numpy(t).cuda()).cpu().numpy()
    _, ref = omlp.mse_grad(flat, f.astype(np.float64), t.astype(np.float64), energy_weight=True)
    cos = float(g @ ref / (np.linalg.norm(g) * np.linalg.norm(ref)))
    assert cos > 0.999, cos
    o = 0
    for name, shape in omlp.SIZES:
        k = int(np.prod(shape))
        gg, rr = g[o:o + k], ref[o:o + k]
        assert np.abs(gg - rr).max() <= 2e-2 * np.abs(rr).max() + 1e-12, name
        o += k


def test_mlp_backward_matches_oracle(sr):
    # the vector-Jacobian product of the backward pass: d(sum dout * y)/dparams
    flat = omlp.bf16_round(omlp.init(7))
    net = sr.Mlp(flat.astype(np.float32))
    rng = np.random.default_rng(4)
    M = 3001
    f = rng.uniform(-1.2, 1.2, (M, 2)).astype(np.float32)
    dout = rng.normal(0.0, 1.0, M).astype(np.float32)
    _say("mlp backward 3001")
    g = net.backward(torch.from_numpy(f), torch.from_numpy(dout)).cpu().numpy()
    ref = omlp.backward(flat, f.astype(np.float64), dout.astype(np.float64))
    cos = float(g @ ref / (np.linalg.norm(g) * np.linalg.norm(ref)))
    assert cos > 0.999, cos
    o = 0
    for name, shape in omlp.SIZES:
        k = int(np.prod(shape))
        gg, rr = g[o:o + k], ref[o:o + k]
        assert np.abs(gg - rr).max() <= 2e-2 * np.abs(rr).max() + 1e-12, name
        o += k


TRAIN_STEPS = 150_000


@pytest.fixture(scope="module")
def trained(sr, table):
    net = sr.Mlp(omlp.init(11).astype(np.float32))
    feats, target = net.make_batch(table, 0xE7A1, 0, 1 << 16)
    w = torch.exp2(target) / (8.0 / (15.0 * math.sqrt(3.0)))
    y0 = net.forward(feats)
    loss0 = float((w * (y0 - target) ** 2).mean())
    _say(f"mlp training {TRAIN_STEPS} x 65536")
    import time
    t0 = time.perf_counter()
    net.train(table, steps=TRAIN_STEPS, batch=1 << 16, lr=2e-3)
    torch.cuda.synchronize()
    print(f"mlp training: {time.perf_counter() - t0:.2f} s for {TRAIN_STEPS} x 65536 samples",
          flush=True)
    torch.cuda.synchronize()
    y1 = net.forward(feats)
    loss1 = float((w * (y1 - target) ** 2).mean())
    _say("mlp judge")
    err = net.judge(table)
    print(f"mlp: loss {loss0:.3e} -> {loss1:.3e}; spectrum error per chi bin "
          f"min {err.min():.2e} median {np.median(err):.2e} max {err.max():.2e}; "
          f"bins on the table {int((err > 1e-3).sum())}/{err.size}", flush=True)
    return net, loss0, loss1, err


def test_table_sampler_against_oracle_inverse_cdf(sr, table, oracle):
    # the table sampler (the surrogate's judge and fallback) against the oracle's
    # inverse number-CDF, with and without the kinematic cut
    rng = np.random.default_rng(12)
    n = 600
    a = rng.integers(0, 2 ** 32, size=n, dtype=np.uint64).astype(np.uint32)
    chi = (10.0 ** rng.uniform(-4.0, 1.5, n)).astype(np.float32)
    u = ((a >> 9).astype(np.float64) + 0.5) / 2 ** 23
    for cut in (False, True):
        _say(f"table sampler vs oracle, cut={cut}")
        x = sr.eval_direct(table, torch.from_numpy(a.view(np.int32)), torch.from_numpy(chi),
                           cut).cpu().numpy().astype(np.float64)
        ref = np.array([oracle.inv_number_cdf(float(c), float(uu), cut)
                        for c, uu in zip(chi.astype(np.float64), u)])
        keep = ref > 1e-5          # below: far under any photon energy that counts
        rel = np.abs(x[keep] / ref[keep] - 1)
        print(f"table sampler cut={cut}: max rel {rel.max():.2e}, median {np.median(rel):.2e}",
              flush=True)
        assert rel.max() <= 2e-5


def test_mlp_training_reduces_loss(trained):
    net, loss0, loss1, err = trained
    assert loss1 < loss0 / 20
    assert np.all(np.isfinite(err))
    # the trained network serves some chi bins within the 1e-3 spectrum bar
    assert (err <= 1e-3).sum() >= 1, err
    assert np.array_equal(net.fallback_host, (err > 1e-3).astype(np.uint8))


def test_judge_matches_host_binning(sr, table, trained):
    """The library's judge against the same statistic computed here from the
    two samplers' x on the judge's grid (sr_eval_direct, sr_mlp_forward) and
    numpy histograms."""
    net, _, _, err = trained
    n_u, cpb, nbx, lo, hi = 1 << 12, 4, 64, 1e-4, 16.4
    err_dev = net.judge(table, n_u=n_u, chi_per_bin=cpb)
    nb = 24
    m = ((np.arange(n_u) + 0.5) * (2 ** 23 / n_u)).astype(np.uint64)
    words = (m << np.uint64(9)).astype(np.uint32)
    u = (2.0 * m.astype(np.float64) + 1.0) * 2.0 ** -24
    lchi = (-4.0 + 0.25 * (np.arange(nb)[:, None] + (np.arange(cpb)[None, :] + 0.5) / cpb))
    lchi = lchi.astype(np.float32).reshape(-1)
    L_ = np.repeat(lchi, n_u)
    chi = torch.from_numpy(np.exp2(L_ * np.float32(3.3219280948873623)).astype(np.float32))
    x_tab = sr.eval_direct(table, torch.from_numpy(np.tile(words, lchi.size).view(np.int32)), chi,
                           True).cpu().numpy().astype(np.float64).reshape(nb, -1)
    f0 = ((L_ + np.float32(1.0)) * np.float32(1.0 / 3.0)).astype(np.float32)
    f1 = np.tile(((np.log2(u) - np.log2(1 - u)) * (math.log(2) / 16)).astype(np.float32), lchi.size)
    y = net.forward(torch.from_numpy(np.stack([f0, f1], 1))).cpu().numpy()
    x_net = np.exp2(y.astype(np.float64)).reshape(nb, -1)
    edges = np.geomspace(lo, hi, nbx + 1)
    ref = np.zeros(nb)
    for b in range(nb):
        ht, _ = np.histogram(x_tab[b], bins=edges, weights=x_tab[b])
        hn, _ = np.histogram(x_net[b], bins=edges, weights=x_net[b])
        ref[b] = np.abs(hn - ht).sum() / ht.sum()
    # the host recomputes the same statistic; FP32 features may differ by an ulp
    np.testing.assert_allclose(err_dev, ref, rtol=0.05, atol=2e-5)
    net.judge(table)    # restore the map of the default judge


def test_step_mlp_sampler_against_oracle(sr, table, oracle, trained):
    net, _, _, err = trained
    cfg = synth.config("c1", b0=(0.0, 0.0, 40.0), gamma_range=(1e3, 1e4))
    n, K, seed, step = 3000, 2, 77, 3
    st = synth.gen_particles(cfg, n=n)
    orc = {k: (v.astype(np.float64) if v.dtype != np.uint32 else v.copy()) for k, v in st.items()}
    orc["x"] = orc["y"] = orc["z"] = None
    ph_o, led_o, det = oracle.step(orc, oracle.Field(0, b0=cfg.b0), cfg.dt, seed, step,
                                   hbar_n=cfg.hbar_n, alpha=cfg.alpha, n_samples=K,
                                   sampler=oracle.SAMPLER_DIRECT, kin_cut=True, push_position=False,
                                   detail=True)
    parts = sr.Particles.from_numpy(st, dim=0)
    parts.x = [None, None, None]
    photons = sr.PhotonBuffer(n, K, dim=3)
    ledger = sr.LedgerBuf(1, sr.n_chunks_uniform(n))
    prm = sr.params_struct(cfg.hbar_n, cfg.alpha, K, sampler=2, kin_cut=True, push_position=False,
                           mlp=net)
    _say("step with the MLP sampler")
    sr.gather_push_emit(parts, None, sr.grid_struct(0, b0=cfg.b0), cfg.dt, seed, step, prm, table,
                        photons, ledger, 0)
    torch.cuda.synchronize()
    ph = photons.gather(n)
    key_o = ph_o["parent"].astype(np.int64) * K + ph_o["k"]
    key_g = ph["parent"].astype(np.int64) * K + ph["k"]
    assert ph_o["eps"].size > 40
    # decisions use the same cut rate as the table sampler: identical off threshold
    near = parity.near_threshold(det["dn"], det["bword"])
    row = np.empty(n, np.int64)
    row[orc["id"]] = np.arange(n)
    flips = set(key_o.tolist()) ^ set(key_g.tolist())
    for kk in flips:
        assert near[row[kk // K] * K + kk % K]
    common = np.intersect1d(key_o, key_g)
    io = np.searchsorted(key_o, common)
    og = np.argsort(key_g)
    ig = og[np.searchsorted(key_g[og], common)]
    x_o = det["xs"][row[ph_o["parent"][io]] * K + ph_o["k"][io]]
    unit = 1.5 * det["chi"][row[ph_o["parent"][io]]] * det["gamma_bar"][row[ph_o["parent"][io]]]
    x_g = ph["eps"][ig] / unit
    lchi = np.log10(det["chi"][row[ph_o["parent"][io]]])
    b = np.floor((lchi + 4.0) / 0.25).astype(int)
    on_table = (b < 0) | (b >= 24) | (err[np.clip(b, 0, 23)] > 1e-3)
    rel = np.abs(x_g / x_o - 1.0)
    if on_table.any():
        assert rel[on_table].max() < 1e-4
    if (~on_table).any():
        # the network's own accuracy, bounded by the judge that admitted it
        assert np.median(rel[~on_table]) < 2e-2
    print(f"mlp step: photons {common.size}, on table {int(on_table.sum())}, network "
          f"median rel err {np.median(rel[~on_table]) if (~on_table).any() else float('nan'):.2e}",
          flush=True)


def test_step_network_path_matches_standalone_forward(sr, table, oracle, trained):
    """With the fallback map cleared the emission kernel evaluates the network on
    the matrix cores for every emitted trial; its x must equal the standalone
    forward pass of the same network at the same (chi, u)."""
    net, _, _, err = trained
    saved = net.fallback.clone()
    net.set_fallback(torch.zeros_like(saved))
    try:
        # chi from 5e-4 to 45 (gamma 5 ... 1e4 in B = 200): most chi bins
        cfg = synth.config("c1", b0=(0.0, 0.0, 200.0), gamma_range=(5.0, 1e4))
        n, K, seed, step = 30000, 8, 91, 2
        st = synth.gen_particles(cfg, n=n)
        orc = {k: (v.astype(np.float64) if v.dtype != np.uint32 else v.copy()) for k, v in st.items()}
        orc["x"] = orc["y"] = orc["z"] = None
        _, _, det = oracle.step(orc, oracle.Field(0, b0=cfg.b0), cfg.dt, seed, step, hbar_n=cfg.hbar_n,
                                alpha=cfg.alpha, n_samples=K, sampler=oracle.SAMPLER_DIRECT,
                                kin_cut=True, push_position=False, detail=True)
        parts = sr.Particles.from_numpy(st, dim=0)
        parts.x = [None, None, None]
        photons = sr.PhotonBuffer(n, K, dim=3)
        ledger = sr.LedgerBuf(1, sr.n_chunks_uniform(n))
        prm = sr.params_struct(cfg.hbar_n, cfg.alpha, K, sampler=2, kin_cut=True,
                               push_position=False, mlp=net)
        _say("step through the network")
        sr.gather_push_emit(parts, None, sr.grid_struct(0, b0=cfg.b0), cfg.dt, seed, step, prm,
                            table, photons, ledger, 0)
        torch.cuda.synchronize()
        ph = photons.gather(n)
        assert ph["eps"].size > 100
        row = np.empty(n, np.int64)
        row[orc["id"]] = np.arange(n)
        r = row[ph["parent"]]
        s = r * K + ph["k"].astype(np.int64)
        chi, gb = det["chi"][r], det["gamma_bar"][r]
        x_gpu = ph["eps"] / (1.5 * chi * gb)
        u = det["rp"][s]
        feats = np.stack([(np.log10(chi) + 1.0) / 3.0, (np.log(u) - np.log1p(-u)) / 16.0],
                         1).astype(np.float32)
        y = net.forward(torch.from_numpy(feats)).cpu().numpy().astype(np.float64)
        rel = np.abs(x_gpu / np.exp2(y) - 1.0)
        # chi enters through binary32 on both sides; x is smooth in chi
        assert np.quantile(rel, 0.99) < 1e-4, rel.max()
        # and the network's samples agree with the oracle's exact inverse CDF
        # as the judge said they would: on the chi bins it admitted, the
        # energy-weighted spectrum of these photons (64 log bins of x on
        # [1e-4, 16.4]) within the 1e-3 bar
        x_exact = det["xs"][s]
        rel_x = np.abs(x_gpu / x_exact - 1)
        b = np.floor((np.log10(chi) + 4.0) / 0.25).astype(int)
        admitted = (b >= 0) & (b < 24) & (err[np.clip(b, 0, 23)] <= 1e-3)
        edges = np.geomspace(1e-4, 16.4, 65)
        he, _ = np.histogram(x_exact[admitted], bins=edges, weights=x_exact[admitted])
        hn, _ = np.histogram(x_gpu[admitted], bins=edges, weights=x_gpu[admitted])
        spec = float(np.abs(hn - he).sum() / max(he.sum(), 1e-300))
        print(f"network path: {x_gpu.size} photons, median |x/x_exact - 1| "
              f"{np.median(rel_x):.2e}; admitted bins: {int(admitted.sum())} photons, spectrum "
              f"error vs the oracle {spec:.2e}", flush=True)
        assert admitted.sum() > 1000
        assert np.median(rel_x[admitted]) <= 1e-3
        # The judge bounds the spectrum error on its dense stratified grid
        # (network vs table, and the table follows the oracle's inverse CDF to
        # ~1e-6: test_table_sampler_against_oracle_inverse_cdf); one step's ~10^4
        # photons fill 64 bins sparsely, and the migration across bin edges then
        # cancels less, so the same network reads somewhat higher here.
        assert spec <= 2e-3
    finally:
        net.set_fallback(saved)


def test_sampler_speed_and_spectrum(sr, table, trained):
    """Plain vs surrogate: one emission step of a 3D K=8 slab workload from the
    same state with the S-proposal sampler, the table-direct sampler, the judged
    network (table where the judge sent it) and the network everywhere.  Reports
    the kernel time of each and the network's speed-up; checks that the direct
    samplers take identical decisions, that the judged network's energy spectrum
    matches the table's, and that the S-proposal run agrees within its
    Monte-Carlo noise."""
    net, _, _, err = trained
    cfg = synth.config("c3", n_particles=1 << 20, grid=(384, 128, 128),
                       momentum="loguniform_gamma", gamma_range=(10.0, 2000.0))
    n, K = cfg.n_particles, cfg.n_samples
    grid = sr.grid_struct(3, n=cfg.grid, dx=(cfg.dx,) * 3)
    fields = sr.Fields(ncells=int(np.prod(cfg.grid)))
    sr.standing_wave(fields, grid, cfg.a0, 0.3)
    st = synth.gen_particles(cfg)
    init = sr.Particles.from_numpy(st, dim=3)
    sorted_ = init.empty_like()
    tile = (16, 4, 4)
    sr.sort_particles(init, sorted_, grid, tile, sr.sort_work(grid, tile, n))
    parts = init.empty_like()
    photons = sr.PhotonBuffer(n, K, dim=3)
    ledger = sr.LedgerBuf(1, sr.n_chunks_uniform(n))
    bins, lo, hi = 64, 1e-8, 1e5
    hwork = sr.hist_work(bins)
    saved = net.fallback.clone()
    variants = [("s_proposal", 0, None), ("table_direct", 1, None), ("mlp_direct", 2, saved),
                ("mlp_network", 2, torch.zeros_like(saved))]
    res = {}
    try:
        for name, sampler, fb in variants:
            if fb is not None:
                net.set_fallback(fb)
            prm = sr.params_struct(cfg.hbar_n, cfg.alpha, K, sampler, cfg.recoil, 0, cfg.kin_cut,
                                   True, mlp=net if sampler == 2 else None)
            times = []
            for rep in range(4):
                for a, b in zip(parts.x + parts.p + [parts.w, parts.id],
                                sorted_.x + sorted_.p + [sorted_.w, sorted_.id]):
                    a.copy_(b)
                ledger.rows.zero_()
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                _say(f"sampler {name} rep {rep}")
                e0.record()
                sr.gather_push_emit(parts, fields, grid, cfg.dt, 99, 5, prm, table, photons,
                                    ledger, 0)
                e1.record()
                torch.cuda.synchronize()
                times.append(e0.elapsed_time(e1))
            hist = torch.zeros(2 * bins, device="cuda", dtype=torch.float64)
            sr.spectrum_histogram(photons, n, lo, hi, bins, hist, hwork)
            row = ledger.row(0)
            res[name] = {"ms": min(times[1:]), "photons": row[5], "emitted": row[0],
                         "ll": row[1], "hist": hist[:bins].cpu().numpy()}
    finally:
        net.set_fallback(saved)
    ref = res["table_direct"]
    for name, r in res.items():
        r["spec_err"] = float(np.abs(r["hist"] - ref["hist"]).sum() / ref["hist"].sum())
    print("samplers (1M electrons, K=8, 384x128x128): " + "; ".join(
        f"{k} {v['ms']:.3f} ms ({ref['ms'] / v['ms']:.2f}x table, "
        f"{res['s_proposal']['ms'] / v['ms']:.2f}x S), {v['photons']:.0f} photons, "
        f"spectrum error vs table {v['spec_err']:.1e}" for k, v in res.items()), flush=True)
    info = table.info()
    tab_bytes = 16 * info.f_pieces + 16 * info.t1_pieces + 8 * info.r_nodes
    print(f"surrogate storage: {2 * 8577} B of bfloat16 weights vs {tab_bytes} B of tables",
          flush=True)
    assert ref["photons"] > 1e5
    # the decision of a direct sampler does not depend on x: identical counts
    assert res["mlp_network"]["photons"] == ref["photons"]
    assert res["mlp_direct"]["photons"] == ref["photons"]
    assert res["mlp_direct"]["spec_err"] <= 1e-3
    # the S proposal draws different numbers: agreement within Monte-Carlo noise
    assert res["s_proposal"]["emitted"] == pytest.approx(ref["emitted"], rel=2e-2)
    assert res["s_proposal"]["ll"] == pytest.approx(ref["ll"], rel=1e-6)
