#!/usr/bin/env python3
"""Throughput of the synchrotron-emission step on one MI355X.

A step is one pass of the whole hot path over the particle ensemble:
  standing-wave field at t^n on the Yee grid (stand-in for the PIC field solve),
  tile sort of the particles every --sort-every steps (gather locality),
  gather + Boris + H_eff + Monte-Carlo emission + photon append + recoil +
  position push (sr_gather_push_emit), the FP64 energy ledger reduction, and
  the photon-spectrum histogram that drains the photon buffer.
`value` is particle-steps/s over the timed steps (wall clock between device
synchronisations).  The emission kernel is also timed alone with HIP events on
the stream it runs on, for the roofline figure.  The CPU baseline is the FP64
oracle on a bounded sample of the same workload.

Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import synth  # noqa: E402

METRIC = "particle-steps/s with emission (plain vs surrogate) at ≤1e-3 spectrum error"
HBM_PEAK_GBS = 8000.0
SPEC_BINS, SPEC_LO, SPEC_HI = 64, 1e-8, 1e5


def photon_bytes(dim: int) -> int:
    # eps, w, dir[3], pos[dim], parent (4 B each) + k (1 B)
    return 4 * (2 + 3 + (2 if dim == 2 else 3) + 1) + 1


def particle_bytes(dim: int) -> tuple[int, int]:
    nd = 2 if dim == 2 else (3 if dim == 3 else 0)
    read = 4 * (nd + 3 + 1 + 1)   # x, p, w, id
    write = 4 * (nd + 3)          # x, p
    return read, write


def energy_hist(eps, w, edges):
    h, _ = np.histogram(np.asarray(eps, np.float64), bins=edges,
                        weights=np.asarray(w, np.float64) * np.asarray(eps, np.float64))
    return h


def run(args):
    import torch

    from paper_1409_5574_amd import api
    from paper_1409_5574_amd import _lib as L

    if not torch.cuda.is_available():
        raise SystemExit("bench.py needs a GPU (HIP device) -- none visible")
    torch.cuda.set_device(0)
    cfg = synth.config(args.config)
    if cfg.dim not in (2, 3) or cfg.sampler != 0:
        raise SystemExit(f"bench workload {args.config}: only the grid S-sampler workloads are timed")
    n = cfg.n_particles
    K = cfg.n_samples
    dim = cfg.dim
    grid = api.grid_struct(dim, n=cfg.grid, dx=(cfg.dx,) * 3)
    ncells = int(np.prod(cfg.grid[:dim]))
    tile = tuple(int(v) for v in args.tile.split(",")) if args.tile else \
        ((64, 4, 1) if dim == 2 else (16, 4, 4))

    # ---------------- inputs resident in HBM
    st0 = synth.gen_particles(cfg)
    parts = api.Particles.from_numpy(st0, dim=dim)
    alt = parts.empty_like()
    sort_work = api.sort_work(grid, tile, n)
    fields = api.Fields(ncells=ncells)
    table = api.Table()
    photons = api.PhotonBuffer(n, cfg.photons_per_particle, dim=dim)
    total_steps = args.warmup + args.steps + 1
    ledger = api.LedgerBuf(total_steps, api.n_chunks_uniform(n))
    n_chunks = api.n_chunks_uniform(n)
    hist = torch.zeros(2 * SPEC_BINS, device="cuda", dtype=torch.float64)
    hwork = api.hist_work(SPEC_BINS)
    prm = api.params_struct(cfg.hbar_n, cfg.alpha, K, 0, cfg.recoil, 0, cfg.kin_cut, True)
    seed = 0xC0FFEE

    api.standing_wave(fields, grid, cfg.a0, 0.0)
    api.sort_particles(parts, alt, grid, tile, sort_work)
    parts, alt = alt, parts
    torch.cuda.synchronize()

    # ---------------- spectrum check: step 0 from the initial state, kept for the CPU leg
    check = None
    if not args.no_cpu_baseline:
        probe = parts.empty_like()
        for a, b in zip(probe.x + probe.p + [probe.w, probe.id], parts.x + parts.p + [parts.w, parts.id]):
            if a is not None:
                a.copy_(b)
        api.gather_push_emit(probe, fields, grid, cfg.dt, seed, 0, prm, table, photons, ledger, 0)
        torch.cuda.synchronize()
        ph = photons.gather(n)
        sel = ph["parent"] < args.cpu_sample
        check = {"eps": ph["eps"][sel], "w": ph["w"][sel], "count": int(sel.sum())}
        del probe

    structs = {id(parts): api.make_structs(parts, fields, photons, ledger),
               id(alt): api.make_structs(alt, fields, photons, ledger)}
    stream = torch.cuda.current_stream()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for _ in range(args.steps)]
    ev_wave = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
               for _ in range(args.steps)]

    def one_step(i, timed_idx=None):
        nonlocal parts, alt
        t = i * cfg.dt
        if timed_idx is not None:
            ev_wave[timed_idx][0].record(stream)
        api.standing_wave(fields, grid, cfg.a0, t)
        if timed_idx is not None:
            ev_wave[timed_idx][1].record(stream)
        if args.sort_every > 0 and i % args.sort_every == 0:
            api.sort_particles(parts, alt, grid, tile, sort_work)
            parts, alt = alt, parts
        s = structs[id(parts)]
        if timed_idx is not None:
            ev[timed_idx][0].record(stream)
        api.gather_push_emit(parts, fields, grid, cfg.dt, seed, i, prm, table, photons, ledger,
                             None, structs=s)
        if timed_idx is not None:
            ev[timed_idx][1].record(stream)
        api.ledger_reduce(ledger, n_chunks, i, s[4])
        api.spectrum_histogram(photons, n, SPEC_LO, SPEC_HI, SPEC_BINS, hist, hwork)

    for i in range(1, args.warmup + 1):
        one_step(i)
    torch.cuda.synchronize()
    hist.zero_()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for j in range(args.steps):
        one_step(args.warmup + 1 + j, j)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0

    k1_ms = np.array([a.elapsed_time(b) for a, b in ev])
    k9_ms = np.array([a.elapsed_time(b) for a, b in ev_wave])
    rows = ledger.rows.cpu().numpy()[args.warmup + 1: args.warmup + 1 + args.steps]
    status = ledger.read_status()
    photons_per_step = rows[:, L.SR_LED_PHOTONS].mean()
    rd, wr = particle_bytes(dim)
    # particles read + written, every grid value once, photon records, segment
    # counts and the per-block (4 chunks) ledger partial rows
    bytes_per_launch = (n * (rd + wr) + 6 * 4 * ncells + photons_per_step * photon_bytes(dim)
                        + n_chunks * 4 + -(-n_chunks // 4) * 8 * L.SR_LEDGER_COLS)
    k1_mean = float(k1_ms.mean())
    achieved = bytes_per_launch / (k1_mean * 1e-3) / 1e9

    value = n * args.steps / wall
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "particle-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": wall * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"{cfg.name}: {cfg.grid[0]}x{cfg.grid[1]}"
                               + (f"x{cfg.grid[2]}" if dim == 3 else "")
                               + f" Yee grid, standing wave a0={cfg.a0:g}, {n} electrons, "
                               f"K={K} trials/step, photon buffer {cfg.photons_per_particle}/particle, "
                               f"S-proposal sampler",
                   "particles": n, "grid": list(cfg.grid[:dim]), "trials_per_step": K,
                   "dt": cfg.dt, "sort_every": args.sort_every, "tile": list(tile[:dim])},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                     "kernel": "push_emit_kernel<float,%d,%d,0>" % (dim, 1 if K <= 1 else K),
                     "kernel_ms": k1_mean, "algorithmic_bytes_per_launch": bytes_per_launch},
        "push_emit_particle_steps_per_s": n / (k1_mean * 1e-3),
        "field_refresh_ms": float(k9_ms.mean()),
        "photons_per_step": float(photons_per_step),
        "ledger_emitted_over_ll": float(rows[:, 0].sum() / max(rows[:, 1].sum(), 1e-300)),
        "chi_max": float(rows[:, L.SR_LED_CHI_MAX].max()),
        "status_bits": int(status),
    }
    if check is not None:
        out["cpu_baseline"], out["spectrum_check"] = cpu_leg(cfg, st0, check, seed, args)
    return out


def cpu_leg(cfg, st0, check, seed, args):
    """The FP64 oracle on the first `cpu_sample` ids: timed for about
    --cpu-seconds, and compared on step 0 with the GPU's photons of those ids."""
    from oracle import oracle as O

    m = args.cpu_sample
    sub = {k: (v[:m].astype(np.float64) if v.dtype != np.uint32 else v[:m].copy())
           for k, v in st0.items()}
    if cfg.dim == 2:
        sub["z"] = None
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    kw = dict(hbar_n=cfg.hbar_n, alpha=cfg.alpha, n_samples=cfg.n_samples, recoil=cfg.recoil,
              kin_cut=cfg.kin_cut, threads=threads)

    def field_at_step(i):
        E, B = synth.standing_wave_grid(cfg, i * cfg.dt)
        return O.Field(cfg.dim, n=cfg.grid, dx=(cfg.dx,) * 3, E=E, B=B)

    f0 = field_at_step(0)
    t0 = time.perf_counter()
    ph0, led0, _ = O.step(sub, f0, cfg.dt, seed, 0, **kw)
    spent = time.perf_counter() - t0
    steps = 1
    per_step = spent
    target = max(args.cpu_seconds, per_step)
    while spent + per_step <= target and steps < 10000:
        f = field_at_step(steps)
        t0 = time.perf_counter()
        O.step(sub, f, cfg.dt, seed, steps, **kw)
        spent += time.perf_counter() - t0
        steps += 1
    edges = np.geomspace(SPEC_LO, SPEC_HI, SPEC_BINS + 1)
    h_g = energy_hist(check["eps"], check["w"], edges)
    h_o = energy_hist(ph0["eps"], ph0["w"], edges)
    err = float(np.abs(h_g - h_o).sum() / max(h_o.sum(), 1e-300))
    base = {"value": m * steps / spent, "unit": "particle-steps/s", "cores": threads,
            "kind": "oracle",
            "sample": f"{m} of the {cfg.n_particles} electrons (ids 0..{m - 1}), {steps} steps, "
                      f"same grid and fields; FP64 C oracle with OpenMP, {spent:.1f} s"}
    spec = {"step": 0, "particles": m, "photons_gpu": check["count"],
            "photons_oracle": int(ph0["eps"].size), "energy_spectrum_error": err,
            "bins": f"{SPEC_BINS} log bins of photon energy in [{SPEC_LO:g}, {SPEC_HI:g}] mc^2"}
    return base, spec


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--config", default="c2")
    ap.add_argument("--sort-every", type=int, default=10)
    ap.add_argument("--tile", default="", help="sort tile in cells, e.g. 256,1,1")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--cpu-sample", type=int, default=65536)
    ap.add_argument("--copy-ref-mb", type=int, default=0,
                    help="also run one plain device copy of this many MiB (counter reference)")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU: this build has no multi-GPU path "
              "(run with --gpus 1)", file=sys.stderr)
        sys.exit(2)
    if args.copy_ref_mb:
        import torch
        a = torch.empty(args.copy_ref_mb << 18, device="cuda", dtype=torch.float32)
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
    out = run(args)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
