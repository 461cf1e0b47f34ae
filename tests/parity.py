"""Comparison helpers for the GPU-vs-oracle parity tests (test-only code).

Tolerances (stated once, used by every parity test):
  momenta      |p_gpu - p_orc| <= 1e-5 * max(|p_orc|, |p_old|) per step
  photons      decisions identical except near threshold, where the trial's
               |b - dN 2^32| <= 1e-5 dN 2^32 + 1 (FP32 dN carries ~1e-6 relative
               error, so such trials may legitimately flip); energy and weight of
               matched photons within 2e-5 relative
  ledger       emitted / LL / recoil sums within 1e-4 relative of the oracle (plus
               the energy of any near-threshold flip)
"""
from __future__ import annotations

import numpy as np

P_TOL = 1e-5
PH_TOL = 2e-5
LEDGER_TOL = 1e-4
NEAR = 1e-5


def quantum_dn_tol(chi, x):
    """Relative accuracy of the FP32 quantum dN at (chi, x): the table's 3e-6,
    the rounding of xi log2 e, and the rounding of delta = 1.5 chi x (about
    4e-7 relative), which 1 - delta turns into a relative error of xi of
    4e-7 delta/(1 - delta), and Q ~ e^-xi multiplies by xi."""
    chi = np.asarray(chi, np.float64)
    x = np.asarray(x, np.float64)
    d = np.minimum(1.5 * chi * x, 1.0 - 1e-12)
    xi = x / (1.0 - d)
    return 3e-6 + 1e-7 * xi + 6e-7 * (xi + 1.0) * d / (1.0 - d)


def near_threshold(dn, b, tol=None):
    """Trials whose decision may flip between FP32 and FP64 dN (tol: per-trial
    relative accuracy of the FP32 dN, default NEAR)."""
    dn = np.asarray(dn, dtype=np.float64)
    tol = NEAR if tol is None else np.maximum(np.asarray(tol, np.float64), NEAR)
    thr = np.minimum(dn, 1.0) * 2.0 ** 32
    near_b = np.abs(np.asarray(b, dtype=np.float64) - thr) <= tol * thr + 1.0
    near_one = np.abs(dn - 1.0) <= tol
    near_kin = np.zeros_like(near_b)
    return near_b | near_one | near_kin


def compare_step(gpu_state: dict, orc_state: dict, old_state: dict, gpu_ph: dict, orc_ph: dict,
                 det: dict, K: int, box=None, xcut_band=None, dn_tol=None):
    """Compare one step.  Returns a report dict; raises AssertionError on failure.
    dn_tol: optional per-trial relative accuracy of the GPU's dN (oracle order),
    for samplers whose FP32 dN is less accurate than NEAR in places."""
    order_g = np.argsort(gpu_state["id"])
    order_o = np.argsort(orc_state["id"])
    ids = orc_state["id"][order_o]
    assert np.array_equal(gpu_state["id"][order_g], ids)
    n = ids.size

    # -------- decisions
    key_o = orc_ph["parent"].astype(np.int64) * K + orc_ph["k"].astype(np.int64)
    key_g = gpu_ph["parent"].astype(np.int64) * K + gpu_ph["k"].astype(np.int64)
    assert np.unique(key_g).size == key_g.size, "duplicate photon tags on the GPU"
    emit_o = np.zeros(n * K, bool)
    emit_g = np.zeros(n * K, bool)
    # oracle detail arrays are in the oracle's particle order; map id -> row
    pos_of_id = np.empty(int(ids.max()) + 1 if n else 1, np.int64)
    pos_of_id[orc_state["id"]] = np.arange(n)
    slot_o = pos_of_id[orc_ph["parent"]] * K + orc_ph["k"].astype(np.int64)
    slot_g = pos_of_id[gpu_ph["parent"]] * K + gpu_ph["k"].astype(np.int64)
    emit_o[slot_o] = True
    emit_g[slot_g] = True
    mism = emit_o != emit_g
    near = near_threshold(det["dn"], det["bword"], dn_tol)
    if xcut_band is not None:
        near |= xcut_band
    bad = mism & ~near
    assert not bad.any(), f"{bad.sum()} decision mismatches away from threshold " \
                          f"(first slots {np.nonzero(bad)[0][:5]}, dn {det['dn'][bad][:5]})"
    flipped_particles = np.unique(np.nonzero(mism)[0] // K)

    # -------- matched photons
    both = emit_o & emit_g
    go = np.full(n * K, -1, np.int64)
    gg = np.full(n * K, -1, np.int64)
    go[slot_o] = np.arange(slot_o.size)
    gg[slot_g] = np.arange(slot_g.size)
    io, ig = go[both], gg[both]
    if io.size:
        rel_e = np.abs(gpu_ph["eps"][ig] - orc_ph["eps"][io]) / np.abs(orc_ph["eps"][io])
        rel_w = np.abs(gpu_ph["w"][ig] - orc_ph["w"][io]) / np.abs(orc_ph["w"][io])
        ddir = np.abs(gpu_ph["dir"][ig] - orc_ph["dir"][io]).max()
        w_tol = PH_TOL if dn_tol is None else PH_TOL + np.asarray(dn_tol)[np.nonzero(both)[0]]
        assert (rel_w <= w_tol).all(), f"photon weight rel err {rel_w.max()}"
        assert rel_e.max() <= PH_TOL, f"photon energy rel err {rel_e.max()} at {np.argmax(rel_e)}"
        assert ddir <= 1e-5, f"photon direction err {ddir}"
    else:
        rel_e = rel_w = np.zeros(1)

    # -------- momenta (particles without a flipped decision)
    keep = np.ones(n, bool)
    keep[flipped_particles] = False
    pg = np.stack([gpu_state[k][order_g] for k in ("px", "py", "pz")], 1)
    po = np.stack([orc_state[k][order_o] for k in ("px", "py", "pz")], 1)
    # a push that is not finite (a non-finite field value or momentum) must be
    # so on both sides; such particles are compared by that alone
    fin_g = np.isfinite(pg).all(1)
    fin_o = np.isfinite(po).all(1)
    assert np.array_equal(fin_g, fin_o), \
        f"non-finite momenta differ: gpu {int((~fin_g).sum())} oracle {int((~fin_o).sum())}"
    pg = np.where(fin_o[:, None], pg, 0.0)
    po = np.where(fin_o[:, None], po, 0.0)
    p_old = np.stack([old_state[k][np.argsort(old_state["id"])] for k in ("px", "py", "pz")], 1)
    den = np.maximum(np.linalg.norm(po, axis=1), np.linalg.norm(p_old, axis=1))
    den = np.maximum(den, 1e-30)
    perr = np.linalg.norm(pg - po, axis=1) / den
    # the orc order and old order agree by id; keep mask is in oracle row order
    keep_sorted = keep[np.argsort(orc_state["id"])] if n else keep
    keep_sorted = keep_sorted & fin_o
    worst = float(perr[keep_sorted].max()) if keep_sorted.any() else 0.0
    assert worst <= P_TOL, f"momentum rel err {worst} (particle {np.argmax(perr * keep_sorted)})"

    # -------- positions (periodic difference; FP32 rounding of x dominates)
    pos_worst = 0.0
    if box is not None:
        for a, k in enumerate(("x", "y", "z")):
            if gpu_state.get(k) is None or orc_state.get(k) is None or a >= len(box):
                continue
            L = box[a]
            d = gpu_state[k][order_g] - orc_state[k][order_o]
            d = (d + L / 2) % L - L / 2
            err = np.abs(d)[keep_sorted]
            lim = 4 * float(np.spacing(np.float32(L))) + 1e-6
            pos_worst = max(pos_worst, float(err.max()) if err.size else 0.0)
            assert (err <= lim).all(), f"position {k} err {err.max()} > {lim}"
    return {"n": n, "photons_oracle": int(emit_o.sum()), "photons_gpu": int(emit_g.sum()),
            "decision_flips": int(mism.sum()), "near_threshold": int(near.sum()),
            "p_rel_err": worst, "eps_rel_err": float(rel_e.max()), "w_rel_err": float(rel_w.max()),
            "pos_err": pos_worst, "flipped_particles": flipped_particles,
            "nonfinite": int((~fin_o).sum())}


def compare_ledger(led_gpu, led_orc, flips_energy: float = 0.0, cols=(0, 1, 2, 3, 4)):
    """Ledger columns against the oracle: emitted, LL and recoil within
    LEDGER_TOL relative (plus the energy of near-threshold flips).  Clamped
    (col 3) is a difference w (delta - |p|) of two rounded quantities, so its
    budget adds the rounding of its terms: delta carries the photon-energy
    tolerance PH_TOL (or the LL loss's), bounded over the clamped particles by
    the step's emitted and LL energy.  Dropped (col 4) is exactly 0 on both
    sides unless the photon buffer overflowed."""
    out = {}
    for c in cols:
        ref = led_orc[c]
        scale = max(abs(ref), 1e-300)
        err = abs(led_gpu[c] - ref)
        out[c] = err / scale
        budget = LEDGER_TOL * scale + flips_energy * (1 + 1e-6) + 1e-12
        if c == 3:
            budget += 2 * PH_TOL * (abs(led_orc[0]) + abs(led_orc[1]))
        assert err <= budget, f"ledger col {c}: gpu {led_gpu[c]} oracle {ref} rel {err / scale}"
    return out
