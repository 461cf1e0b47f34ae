"""The emission step that allocates nothing (sr_gather_push_emit_noalloc)
against the step with a caller workspace (sr_gather_push_emit followed by
sr_ledger_reduce): the same particles, photons, ledger row and status, on two
calls in a row, the second with a smaller input (the library's device array
keeps the first call's contents)."""
from __future__ import annotations

import sys

import numpy as np
import pytest

import synth

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


def _one(sr, table, cfg, st, fields, grid, prm, seed, step, noalloc):
    n = st["px"].size
    parts = sr.Particles.from_numpy(st, dim=3)
    photons = sr.PhotonBuffer(n, cfg.photons_per_particle, dim=3)
    if noalloc:
        row = torch.full((8,), 7.0, device="cuda", dtype=torch.float64)
        status = torch.zeros(1, device="cuda", dtype=torch.int32)
        sr.gather_push_emit_noalloc(parts, fields, grid, cfg.dt, seed, step, prm, table, photons,
                                    row, status)
        torch.cuda.synchronize()
        led, stat = row.cpu().numpy(), int(status.item())
    else:
        ledger = sr.LedgerBuf(1, sr.n_chunks_uniform(n))
        sr.gather_push_emit(parts, fields, grid, cfg.dt, seed, step, prm, table, photons, ledger, 0)
        torch.cuda.synchronize()
        led, stat = ledger.row(0), ledger.read_status()
    return parts.to_numpy(), photons.gather(n), led, stat


def test_noalloc_step_matches_workspace_step(sr):
    table = sr.Table()
    cfg = synth.config("c3", grid=(64, 48, 40), slab=None)
    grid = sr.grid_struct(3, n=cfg.grid, dx=(cfg.dx,) * 3)
    E, B = synth.standing_wave_grid(cfg, 0.4)
    fields = sr.Fields(E, B)
    prm = sr.params_struct(cfg.hbar_n, cfg.alpha, cfg.n_samples, recoil=cfg.recoil,
                           kin_cut=cfg.kin_cut)
    # 300 000 particles: 1172 partial rows, summed in two levels; then 20 000:
    # 79 rows, one level, over the first call's leftovers
    for n, seed in ((300_000, 31), (20_000, 32)):
        st = synth.gen_particles(cfg, n=n, seed=seed)
        for k in ("px", "py", "pz"):
            st[k] = (st[k].astype(np.float64) * 3000.0).astype(np.float32)
        _say(f"noalloc step n={n}")
        ref = _one(sr, table, cfg, st, fields, grid, prm, 77, 5, noalloc=False)
        got = _one(sr, table, cfg, st, fields, grid, prm, 77, 5, noalloc=True)
        (pa, pha, la, sa), (pb, phb, lb, sb) = ref, got
        for k in ("x", "y", "z", "px", "py", "pz"):
            assert np.array_equal(pa[k], pb[k]), k
        assert pha["count"] == phb["count"] > 1000
        for k in ("eps", "w", "dir", "pos", "parent", "k"):
            assert np.array_equal(pha[k], phb[k]), k
        assert np.array_equal(la, lb)
        assert la[5] == pha["count"]
        assert sa == sb
    # sizes beyond the library's array are refused before any launch
    import ctypes as C
    L = sr.L
    small = sr.Particles.from_numpy(synth.gen_particles(cfg, n=64), dim=3)
    ps = small.struct()
    ps.n = (L.SR_NOALLOC_MAX_CHUNKS + 1) * L.SR_CHUNK
    cs = L.Chunking(L.SR_NOALLOC_MAX_CHUNKS + 1, None)
    fs = fields.struct()
    phs = sr.PhotonBuffer(64, 1, dim=3).struct()
    row = torch.zeros(8, device="cuda", dtype=torch.float64)
    status = torch.zeros(1, device="cuda", dtype=torch.int32)
    rc = sr.lib().sr_gather_push_emit_noalloc(C.byref(ps), C.byref(fs), C.byref(grid), cfg.dt, 1,
                                              0, C.byref(prm), table.handle, C.byref(cs),
                                              C.byref(phs), row.data_ptr(), status.data_ptr(),
                                              None)
    assert rc == L.SR_E_UNSUPPORTED
    table.free()
