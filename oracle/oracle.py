"""Python side of the FP64 CPU oracle (test infrastructure only).

The arithmetic lives in ``sr_oracle.c`` (plain C99, FP64); this module loads it
with ctypes and adds the pieces that are plain numpy: the binned-spectrum
metric, the inverse-CDF table check and the FP64 MLP used to check the
surrogate's gradients.  Only the test suite, the smoke check and the
CPU-baseline leg of the benchmark import it.  It imports nothing from the HIP
package.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libsr_oracle.so")
SRC_PATH = os.path.join(_HERE, "sr_oracle.c")

FIELD_ANALYTIC, FIELD_2D, FIELD_3D = 0, 2, 3
RECOIL_NONE, RECOIL_PHOTON, RECOIL_LL = 0, 1, 2
DN_WEIGHT, DN_CLAMP = 0, 1
SAMPLER_S, SAMPLER_DIRECT, SAMPLER_QUANTUM = 0, 1, 2


def build(force: bool = True) -> str:
    """Compile sr_oracle.c with gcc (IEEE FP64, no fast-math, no contraction)."""
    stale = (not os.path.exists(LIB_PATH)
             or os.path.getmtime(LIB_PATH) < max(os.path.getmtime(SRC_PATH),
                                                 os.path.getmtime(SRC_PATH[:-1] + "h")))
    if force or stale:
        cmd = ["gcc", "-O2", "-std=c99", "-D_DEFAULT_SOURCE", "-ffp-contract=off",
               "-fopenmp", "-Wall", "-shared", "-fPIC", "-o", LIB_PATH, SRC_PATH, "-lm"]
        subprocess.run(cmd, check=True)
    return LIB_PATH


class _Field(C.Structure):
    _fields_ = [("kind", C.c_int32), ("n", C.c_int64 * 3), ("dx", C.c_double * 3),
                ("origin", C.c_double * 3), ("e0", C.c_double * 3), ("b0", C.c_double * 3),
                ("E", C.c_void_p * 3), ("B", C.c_void_p * 3)]


class _Params(C.Structure):
    _fields_ = [("hbar_n", C.c_double), ("alpha", C.c_double), ("n_samples", C.c_int32),
                ("recoil", C.c_int32), ("dn_policy", C.c_int32), ("kin_cut", C.c_int32),
                ("sampler", C.c_int32), ("push_position", C.c_int32), ("omega_grid", C.c_double)]


class _Photons(C.Structure):
    _fields_ = [("capacity", C.c_int64), ("count", C.c_int64), ("eps", C.c_void_p),
                ("w", C.c_void_p), ("dir", C.c_void_p), ("pos", C.c_void_p),
                ("parent", C.c_void_p), ("k", C.c_void_p)]


class _Detail(C.Structure):
    _fields_ = [("heff", C.c_void_p), ("gamma_bar", C.c_void_p), ("chi", C.c_void_p),
                ("ratio", C.c_void_p), ("dn", C.c_void_p), ("xs", C.c_void_p),
                ("rp", C.c_void_p), ("bword", C.c_void_p), ("emit", C.c_void_p)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        build(force=False)
        L = C.CDLL(LIB_PATH)
        d, p, i64, i32, u64 = C.c_double, C.c_void_p, C.c_int64, C.c_int32, C.c_uint64
        L.orc_synchrotron_F.restype = d
        L.orc_synchrotron_F.argtypes = [d, d]
        L.orc_synchrotron_F_array.argtypes = [i64, p, p, d]
        L.orc_number_integral.restype = d
        L.orc_number_integral.argtypes = [d, d]
        L.orc_energy_integral.restype = d
        L.orc_energy_integral.argtypes = [d, d]
        L.orc_inv_number_cdf.restype = d
        L.orc_inv_number_cdf.argtypes = [d, d, i32]
        L.orc_proposal_a.restype = d
        L.orc_proposal_Pa_f32.restype = d
        L.orc_proposal_invert.argtypes = [d, d, p, p]
        L.orc_trial_dn.restype = d
        L.orc_trial_dn.argtypes = [d, d, d, d, p]
        L.orc_bessel_K.restype = d
        L.orc_bessel_K.argtypes = [d, d, d]
        L.orc_bessel_K_tail.restype = d
        L.orc_bessel_K_tail.argtypes = [d, d, d]
        L.orc_quantum_kernel.restype = d
        L.orc_quantum_kernel.argtypes = [d, d, d]
        L.orc_quantum_kernel_array.argtypes = [i64, p, p, p, d]
        L.orc_trial_dn_quantum.restype = d
        L.orc_trial_dn_quantum.argtypes = [d, d, d, d, p]
        L.orc_boris.argtypes = [p, p, p, d, d, p]
        L.orc_heff.restype = d
        L.orc_heff.argtypes = [p, p, d, p, p]
        L.orc_gather.argtypes = [C.POINTER(_Field), p, p, p]
        L.orc_philox_array.argtypes = [i64, p, p, p]
        L.orc_step.restype = C.c_int
        L.orc_step.argtypes = [i64, p, p, p, p, p, p, p, p, C.POINTER(_Field), d, u64, u64,
                               C.POINTER(_Params), C.POINTER(_Photons), p, C.POINTER(_Detail), i32]
        _lib = L
    return _lib


def _ptr(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


# ---------------------------------------------------------------- primitives
def synchrotron_F(x, h: float = 0.1) -> np.ndarray:
    x = np.ascontiguousarray(np.atleast_1d(np.asarray(x, dtype=np.float64)))
    out = np.empty_like(x)
    lib().orc_synchrotron_F_array(x.size, _ptr(x), _ptr(out), h)
    return out


def number_integral(x: float, h: float = 0.1) -> float:
    return lib().orc_number_integral(float(x), h)


def energy_integral(x: float, h: float = 0.1) -> float:
    return lib().orc_energy_integral(float(x), h)


def inv_number_cdf(chi: float, u: float, kin_cut: bool) -> float:
    return lib().orc_inv_number_cdf(float(chi), float(u), int(bool(kin_cut)))


def bessel_K(nu: float, xi: float, h: float = 0.1) -> float:
    return lib().orc_bessel_K(float(nu), float(xi), h)


def bessel_K_tail(nu: float, xi: float, h: float = 0.1) -> float:
    return lib().orc_bessel_K_tail(float(nu), float(xi), h)


def quantum_kernel(x, chi, h: float = 0.1) -> np.ndarray:
    """Q(x, chi), the quantum-corrected counterpart of F(x)/x (broadcasts)."""
    xb, cb = np.broadcast_arrays(np.asarray(x, np.float64), np.asarray(chi, np.float64))
    xb = np.ascontiguousarray(xb.ravel())
    cb = np.ascontiguousarray(cb.ravel())
    out = np.empty_like(xb)
    lib().orc_quantum_kernel_array(xb.size, _ptr(xb), _ptr(cb), _ptr(out), h)
    return out


def trial_dn_quantum(Rp: float, rate: float, chi: float, Pa: float | None = None):
    """dN of one quantum trial at uniform R' (returns (dN, x))."""
    if Pa is None:
        Pa = proposal_Pa_f32()
    x = C.c_double()
    dn = lib().orc_trial_dn_quantum(float(Rp), float(Pa), float(rate), float(chi), C.byref(x))
    return dn, x.value


def proposal_a() -> float:
    return lib().orc_proposal_a()


def proposal_Pa_f32() -> float:
    return lib().orc_proposal_Pa_f32()


def proposal_invert(Rp: float, Pa: float | None = None):
    if Pa is None:
        Pa = proposal_Pa_f32()
    x, S = C.c_double(), C.c_double()
    lib().orc_proposal_invert(float(Rp), float(Pa), C.byref(x), C.byref(S))
    return x.value, S.value


def trial_dn(Rp: float, rate: float, xcut: float = float("inf"), Pa: float | None = None):
    """dN of one trial at uniform R' (returns (dN, x))."""
    if Pa is None:
        Pa = proposal_Pa_f32()
    x = C.c_double()
    dn = lib().orc_trial_dn(float(Rp), float(Pa), float(rate), float(xcut), C.byref(x))
    return dn, x.value


def boris(p, E, B, q: float, dt: float) -> np.ndarray:
    p, E, B = (np.ascontiguousarray(v, dtype=np.float64) for v in (p, E, B))
    out = np.empty(3)
    lib().orc_boris(_ptr(p), _ptr(E), _ptr(B), q, dt, _ptr(out))
    return out


def heff(p_old, p_new, dt: float):
    """Returns (H_eff, gamma_bar, unclamped dp_perp/p)."""
    a, b = (np.ascontiguousarray(v, dtype=np.float64) for v in (p_old, p_new))
    g, r = C.c_double(), C.c_double()
    H = lib().orc_heff(_ptr(a), _ptr(b), dt, C.byref(g), C.byref(r))
    return H, g.value, r.value


def philox4x32_10(ctr, key) -> np.ndarray:
    """ctr: [n,4] uint32, key: [2] uint32 -> [n,4] uint32."""
    ctr = np.ascontiguousarray(np.atleast_2d(np.asarray(ctr, dtype=np.uint32)))
    key = np.ascontiguousarray(np.asarray(key, dtype=np.uint32))
    out = np.empty_like(ctr)
    lib().orc_philox_array(ctr.shape[0], _ptr(ctr), _ptr(key), _ptr(out))
    return out


# ---------------------------------------------------------------- one step
class Field:
    """Field description for the oracle.  kind: 0 analytic, 2 = 2D, 3 = 3D."""

    def __init__(self, kind, n=(1, 1, 1), dx=(1.0, 1.0, 1.0), origin=(0.0, 0.0, 0.0),
                 e0=(0.0, 0.0, 0.0), b0=(0.0, 0.0, 0.0), E=None, B=None):
        self.kind, self.n, self.dx, self.origin = kind, n, dx, origin
        self.e0, self.b0 = e0, b0
        self.E = None if E is None else [np.ascontiguousarray(a, dtype=np.float32) for a in E]
        self.B = None if B is None else [np.ascontiguousarray(a, dtype=np.float32) for a in B]

    def struct(self) -> _Field:
        f = _Field()
        f.kind = self.kind
        for a in range(3):
            f.n[a] = int(self.n[a])
            f.dx[a] = float(self.dx[a])
            f.origin[a] = float(self.origin[a])
            f.e0[a] = float(self.e0[a])
            f.b0[a] = float(self.b0[a])
            f.E[a] = None if self.E is None else self.E[a].ctypes.data
            f.B[a] = None if self.B is None else self.B[a].ctypes.data
        return f


def gather(field: "Field", pos):
    """(E, B) at one position."""
    pos = np.ascontiguousarray(pos, dtype=np.float64)
    E, B = np.empty(3), np.empty(3)
    fs = field.struct()
    lib().orc_gather(C.byref(fs), _ptr(pos), _ptr(E), _ptr(B))
    return E, B


def step(state: dict, field: Field, dt: float, seed: int, step_index: int, *, hbar_n: float,
         alpha: float, n_samples: int = 1, recoil: int = RECOIL_PHOTON, dn_policy: int = DN_WEIGHT,
         kin_cut: bool = False, sampler: int = SAMPLER_S, push_position: bool = True,
         detail: bool = False, threads: int = 0, omega_grid: float = 0.0):
    """Advance ``state`` (dict of FP64 arrays x,y,z,px,py,pz,w and uint32 id) by one step
    in place.  Returns (photons dict, ledger[5], detail dict or None)."""
    n = int(state["px"].shape[0])
    K = int(n_samples)
    for k in ("px", "py", "pz", "w"):
        assert state[k].dtype == np.float64 and state[k].flags.c_contiguous
    for k in ("x", "y", "z"):
        if state.get(k) is not None:
            assert state[k].dtype == np.float64 and state[k].flags.c_contiguous
    assert state["id"].dtype == np.uint32
    cap = max(n * K, 1)
    ph = {"eps": np.empty(cap), "w": np.empty(cap), "dir": np.empty((cap, 3)),
          "pos": np.empty((cap, 3)), "parent": np.empty(cap, np.uint32), "k": np.empty(cap, np.uint32)}
    phs = _Photons(cap, 0, *(ph[k].ctypes.data for k in ("eps", "w", "dir", "pos", "parent", "k")))
    prm = _Params(hbar_n, alpha, K, recoil, dn_policy, int(bool(kin_cut)), sampler,
                  int(bool(push_position)), float(omega_grid))
    det = None
    dets = None
    if detail:
        det = {"heff": np.empty(n), "gamma_bar": np.empty(n), "chi": np.empty(n),
               "ratio": np.empty(n), "dn": np.empty(n * K), "xs": np.empty(n * K),
               "rp": np.empty(n * K), "bword": np.empty(n * K, np.uint32),
               "emit": np.empty(n * K, np.uint8)}
        dets = _Detail(*(det[k].ctypes.data for k in ("heff", "gamma_bar", "chi", "ratio", "dn",
                                                       "xs", "rp", "bword", "emit")))
    ledger = np.zeros(5)
    fs = field.struct()
    rc = lib().orc_step(n, _ptr(state.get("x")), _ptr(state.get("y")), _ptr(state.get("z")),
                        _ptr(state["px"]), _ptr(state["py"]), _ptr(state["pz"]), _ptr(state["w"]),
                        _ptr(state["id"]), C.byref(fs), dt, seed & 0xFFFFFFFFFFFFFFFF, step_index,
                        C.byref(prm), C.byref(phs), _ptr(ledger),
                        C.byref(dets) if dets is not None else None, threads)
    if rc != 0:
        raise RuntimeError(f"orc_step failed with {rc}")
    m = phs.count
    photons = {k: v[:m] for k, v in ph.items()}
    return photons, ledger, det


# ---------------------------------------------------------------- validity diagnostics
VALID_QUANTUM, VALID_NON_SYNCHROTRON = 1, 2


def validity_flags(heff, chi, tau_em: float) -> np.ndarray:
    """Per-particle flags of the method's two stated limits.

    VALID_QUANTUM: chi >= 1, where the classical emission formula fails and a QED
    treatment is needed (section "Limitations").
    VALID_NON_SYNCHROTRON: 0 < H_eff tau_em <= 1.  The synchrotron (wiggler)
    spectrum needs the field to vary slower than the particle turns by an angle
    1/gamma, tau_em > 1/(gamma omega_H) with omega_H = e H_eff/(m c gamma)
    (section "Synchrotron emission"), i.e. H_eff tau_em > 1 in normalised units."""
    heff = np.asarray(heff, np.float64)
    chi = np.asarray(chi, np.float64)
    f = np.where(chi >= 1.0, VALID_QUANTUM, 0)
    f |= np.where((heff > 0.0) & (heff * tau_em <= 1.0), VALID_NON_SYNCHROTRON, 0)
    return f.astype(np.uint8)


def validity_sums(w, chi, beta2, flags, alpha: float, hbar_n: float, dt: float):
    """{sum w, sum w [quantum], sum w [non-synchrotron], sum w P, sum w P [quantum],
    sum w P [non-synchrotron]} with P = (2/3)(alpha/hbar_n) chi^2 beta^2 dt, the
    Landau-Lifshitz energy of the step (eq:LLformOfRRForce with |v| = beta)."""
    w = np.asarray(w, np.float64)
    P = (2.0 / 3.0) * (alpha / hbar_n) * np.asarray(chi) ** 2 * np.asarray(beta2) * dt
    q = (flags & VALID_QUANTUM) != 0
    ns = (flags & VALID_NON_SYNCHROTRON) != 0
    return np.array([w.sum(), w[q].sum(), w[ns].sum(), (w * P).sum(), (w * P)[q].sum(),
                     (w * P)[ns].sum()])


# ---------------------------------------------------------------- spectrum metric
def spectrum_bins(n_bins: int = 64, x_lo: float = 1e-4, x_hi: float = 16.4) -> np.ndarray:
    """Log-spaced bin edges in x = omega/omega_c for the binned-spectrum metric."""
    return np.geomspace(x_lo, x_hi, n_bins + 1)


def binned_energy_spectrum(x, w_eps, edges) -> np.ndarray:
    """Energy-weighted histogram: sum of w*eps per bin of x."""
    h, _ = np.histogram(np.asarray(x, dtype=np.float64), bins=edges,
                        weights=np.asarray(w_eps, dtype=np.float64))
    return h


def spectrum_error(h, h_ref) -> float:
    """sum |h - h_ref| / sum h_ref."""
    h = np.asarray(h, dtype=np.float64)
    h_ref = np.asarray(h_ref, dtype=np.float64)
    den = h_ref.sum()
    return float(np.abs(h - h_ref).sum() / den) if den > 0 else float(np.abs(h).sum())
