"""The step captured into a HIP graph: several replays, each from the same
restored state with eager work and synchronisations in between, must give what
the eager launches give (field refresh, tile sort, emission step, ledger
reduction, spectrum histogram)."""
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


def _copy(dst, src):
    for a, b in zip(dst.x + dst.p + [dst.w, dst.id], src.x + src.p + [src.w, src.id]):
        if a is not None:
            a.copy_(b)


def _snapshot(cur, ledger, hist, photons, n):
    """State in an order-free form: the tile sort leaves the order inside a tile
    open, so particles are compared by id and photons by (parent, trial)."""
    ids = cur.id.cpu().numpy().view(np.uint32)
    o = np.argsort(ids)
    ph = photons.gather(n)
    key = ph["parent"].astype(np.int64) * 64 + ph["k"].astype(np.int64)
    po = np.argsort(key)
    return {"x": [t.cpu().numpy()[o] for t in cur.x if t is not None],
            "p": [t.cpu().numpy()[o] for t in cur.p],
            "id": ids[o],
            "rows": ledger.rows.cpu().numpy().copy(),
            "hist": hist.cpu().numpy().copy(),
            "ph_key": key[po], "ph_eps": ph["eps"][po], "ph_w": ph["w"][po]}


def test_step_graph_replays_match_eager(sr):
    cfg = synth.config("c2", n_particles=1 << 16, grid=(256, 256, 1))
    n, steps, sort_every, seed = cfg.n_particles, 6, 3, 0x9A4B
    grid = sr.grid_struct(2, n=cfg.grid, dx=(cfg.dx,) * 3)
    tile = (64, 4, 1)
    table = sr.Table()
    init = sr.Particles.from_numpy(synth.gen_particles(cfg), dim=2)
    A, B = init.empty_like(), init.empty_like()
    fields = sr.Fields(ncells=int(np.prod(cfg.grid[:2])))
    photons = sr.PhotonBuffer(n, cfg.photons_per_particle, dim=2)
    n_chunks = sr.n_chunks_uniform(n)
    ledger = sr.LedgerBuf(steps, n_chunks)
    bins = 64
    hist = torch.zeros(2 * bins, device="cuda", dtype=torch.float64)
    hwork = sr.hist_work(bins)
    sw = sr.sort_work(grid, tile, n)
    prm = sr.params_struct(cfg.hbar_n, cfg.alpha, cfg.n_samples, 0, cfg.recoil, 0, cfg.kin_cut, True)
    # a warm start: the field is strong from the first step
    t_off = 0.7

    def run_steps(cur, oth):
        for i in range(steps):
            sr.standing_wave(fields, grid, cfg.a0, t_off + i * cfg.dt)
            if i % sort_every == 0:
                sr.sort_particles(cur, oth, grid, tile, sw)
                cur, oth = oth, cur
            sr.gather_push_emit(cur, fields, grid, cfg.dt, seed, i, prm, table, photons, ledger, None)
            sr.ledger_reduce(ledger, n_chunks, i)
            sr.spectrum_histogram(photons, n, 1e-8, 1e5, bins, hist, hwork)
        return cur

    def reset():
        _copy(A, init)
        hist.zero_()
        ledger.rows.zero_()
        photons.seg_count.zero_()
        torch.cuda.synchronize()

    _say("graph: eager reference")
    reset()
    cur = run_steps(A, B)
    torch.cuda.synchronize()
    ref = _snapshot(cur, ledger, hist, photons, n)
    assert ref["rows"][:, 5].sum() > 100          # photons were emitted

    _say("graph: capture")
    reset()
    g = torch.cuda.CUDAGraph()
    cap = torch.cuda.Stream()
    cap.wait_stream(torch.cuda.current_stream())
    with torch.cuda.graph(g, stream=cap):
        cur_g = run_steps(A, B)
    torch.cuda.synchronize()
    for rep in range(3):
        reset()
        _say(f"graph: replay {rep}")
        g.replay()
        torch.cuda.synchronize()
        got = _snapshot(cur_g, ledger, hist, photons, n)
        for q in range(2):
            assert np.array_equal(got["x"][q], ref["x"][q]), (rep, q)
        for q in range(3):
            assert np.array_equal(got["p"][q], ref["p"][q]), (rep, q)
        assert np.array_equal(got["id"], ref["id"])
        # last step's photons: the same records
        assert np.array_equal(got["ph_key"], ref["ph_key"])
        assert np.array_equal(got["ph_eps"], ref["ph_eps"])
        assert np.array_equal(got["ph_w"], ref["ph_w"])
        # FP64 sums whose order follows the particle order inside a tile: equal
        # to rounding
        np.testing.assert_allclose(got["rows"], ref["rows"], rtol=1e-12, atol=0)
        np.testing.assert_allclose(got["hist"], ref["hist"], rtol=1e-12, atol=0)
    del g
