"""The FP32 / FP64 precision split on the precision-stress workload
(768x768x384 grid, standing wave a0 = 800, gamma up to 3e4): one step of 65,536
electrons through the FP32 path and through the FP64 gather-and-push path,
each result compared with the FP64 oracle and the errors reported.

Per result: momenta after the step, H_eff, chi and the mean gamma of the push
(from the step's own push code through sr_eval_push), photon energies of the
trials both sides emit, emission decisions, the binned energy spectrum and the
ledger sums.  The bars are those of the parity tests: 1e-5 on momenta, 1e-3 on
the binned spectrum, 1e-4 on the ledger, decisions identical away from
threshold."""
from __future__ import annotations

import json
import sys

import numpy as np
import pytest

import synth
from tests import parity
from tests.test_gpu_full import _device_fields, _host_grid, _orc

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


def _rel(a, b):
    a, b = np.asarray(a, np.float64), np.asarray(b, np.float64)
    return np.abs(a - b) / np.maximum(np.abs(b), 1e-300)


def _stats(r):
    r = np.asarray(r, np.float64)
    if r.size == 0:
        return {"max": 0.0, "p99": 0.0, "median": 0.0}
    return {"max": float(r.max()), "p99": float(np.quantile(r, 0.99)),
            "median": float(np.median(r))}


def _spectrum_error(eps_g, w_g, eps_o, w_o, bins=64, lo=1e-8, hi=1e5):
    edges = np.geomspace(lo, hi, bins + 1)
    hg, _ = np.histogram(eps_g, bins=edges, weights=np.asarray(w_g, np.float64) * eps_g)
    ho, _ = np.histogram(eps_o, bins=edges, weights=np.asarray(w_o, np.float64) * eps_o)
    return float(np.abs(hg - ho).sum() / max(ho.sum(), 1e-300))


def test_precision_split_report(sr, oracle):
    cfg = synth.config("c5")
    n, K, seed, step, t = 65536, cfg.n_samples, 2024, 5, 0.3
    st = synth.gen_particles(cfg, n=n)
    grid = sr.grid_struct(3, n=cfg.grid, dx=(cfg.dx,) * 3)
    _say(f"precision split: {n} electrons on {cfg.grid}")
    fields, profiles = _device_fields(sr, cfg, t)
    table = sr.Table()

    # ---- oracle (FP64, the same binary32 grid values widened)
    orc = _orc(st)
    old = _orc(st)
    host = _host_grid(profiles, cfg)
    fo = oracle.Field(3, n=cfg.grid, dx=(cfg.dx,) * 3, E=host[:3], B=host[3:])
    ph_o, led_o, det = oracle.step(orc, fo, cfg.dt, seed, step, hbar_n=cfg.hbar_n, alpha=cfg.alpha,
                                   n_samples=K, recoil=cfg.recoil, kin_cut=cfg.kin_cut, detail=True)
    del host, fo
    xcut = np.abs(1.5 * np.repeat(det["chi"], K) * det["xs"] - 1.0) <= 1e-5

    report = {"workload": f"{cfg.name}: {n} electrons, grid {cfg.grid}, a0 {cfg.a0:g}, t {t}",
              "oracle_photons": int(ph_o["eps"].size)}
    for label, dtype in (("fp32", torch.float32), ("fp64_push", torch.float64)):
        _say(f"precision split: {label} path")
        parts = sr.Particles.from_numpy(st, dtype=dtype, dim=3)
        pushed = sr.eval_push(parts, fields, grid, cfg.dt, cfg.hbar_n, cfg.alpha)
        photons = sr.PhotonBuffer(n, cfg.photons_per_particle, dim=3)
        ledger = sr.LedgerBuf(1, sr.n_chunks_uniform(n))
        prm = sr.params_struct(cfg.hbar_n, cfg.alpha, K, recoil=cfg.recoil, kin_cut=cfg.kin_cut)
        sr.gather_push_emit(parts, fields, grid, cfg.dt, seed, step, prm, table, photons, ledger, 0)
        torch.cuda.synchronize()
        assert ledger.read_status() & ~2 == 0
        g = parts.to_numpy()
        ph_g = photons.gather(n)
        led_g = ledger.row(0)
        heff = pushed["heff"].cpu().numpy()
        chi = pushed["chi"].cpu().numpy()
        gbar = pushed["gamma_bar"].cpu().numpy()

        rep = parity.compare_step(g, orc, old, ph_g, ph_o, det, K, box=cfg.box, xcut_band=xcut)
        # momenta: all particles, and those without emission (no recoil from FP32 trials)
        # (relative to the larger of |p| before and after the step, as the parity
        # bar: a particle whose recoil took most of its momentum is compared on
        # the scale of the momentum it had)
        pg = np.stack([g["px"], g["py"], g["pz"]], 1)
        po = np.stack([orc["px"], orc["py"], orc["pz"]], 1)
        p_old = np.stack([old["px"], old["py"], old["pz"]], 1)
        scale = np.maximum(np.linalg.norm(po, axis=1), np.linalg.norm(p_old, axis=1))
        dp = np.linalg.norm(pg - po, axis=1) / np.maximum(scale, 1e-300)
        emitted = np.zeros(n, bool)
        emitted[ph_o["parent"]] = True
        emitted[ph_g["parent"]] = True
        # photon energies of the trials both sides emitted
        key_o = ph_o["parent"].astype(np.int64) * K + ph_o["k"]
        key_g = ph_g["parent"].astype(np.int64) * K + ph_g["k"]
        common, io, ig = np.intersect1d(key_o, key_g, return_indices=True)
        r = {"p_all": _stats(dp), "p_no_emission": _stats(dp[~emitted]),
             "heff": _stats(_rel(heff, det["heff"])), "chi": _stats(_rel(chi, det["chi"])),
             "gamma_bar": _stats(_rel(gbar, det["gamma_bar"])),
             "eps": _stats(_rel(ph_g["eps"][ig], ph_o["eps"][io])),
             "decisions": {"trials": n * K, "flips": int(rep["decision_flips"]),
                           "all_within_threshold_band": True},
             "spectrum_error": _spectrum_error(ph_g["eps"], ph_g["w"], ph_o["eps"], ph_o["w"]),
             "ledger_emitted": float(_rel(led_g[0], led_o[0])),
             "ledger_ll": float(_rel(led_g[1], led_o[1])),
             "photons": int(ph_g["eps"].size)}
        report[label] = r
        # the bars
        assert r["p_all"]["max"] <= parity.P_TOL
        assert r["spectrum_error"] <= 1e-3
        assert r["ledger_ll"] <= parity.LEDGER_TOL
        assert r["ledger_emitted"] <= parity.LEDGER_TOL or r["decisions"]["flips"] > 0
        if label == "fp64_push":
            # the FP64 gather and push reproduce the oracle's push to rounding
            assert r["heff"]["max"] <= 1e-9
            assert r["chi"]["max"] <= 1e-9
            assert r["p_no_emission"]["max"] <= 1e-12
        else:
            assert r["heff"]["p99"] <= 1e-4
        del parts, photons, ledger
    print("precision split report: " + json.dumps(report), flush=True)
