"""Workload definitions: constants, configurations, particle and field generators."""
from __future__ import annotations

import dataclasses
import math

import numpy as np

# CODATA 2022 values (SI); only used to form the dimensionless parameters below.
ALPHA = 7.2973525643e-3
_M_E = 9.1093837139e-31
_C = 299792458.0
_Q_E = 1.602176634e-19
_HBAR = 1.054571817e-34

_B_CRIT = _M_E ** 2 * _C ** 2 / (_Q_E * _HBAR)          # Schwinger field, tesla
_OMEGA_08UM = 2.0 * math.pi * _C / 0.8e-6                # laser frequency at 0.8 um

# hbar omega_r / (m c^2) for the two choices of omega_r
HBAR_N_1E5T = 1e5 / _B_CRIT                              # omega_r = eB/m at B = 1e5 T
HBAR_N_08UM = _HBAR * _OMEGA_08UM / (_M_E * _C ** 2)     # omega_r = laser frequency

TWO_PI = 2.0 * math.pi

# Yee staggering of the six components, in cells: Ex Ey Ez Bx By Bz
_YEE = ((0.5, 0.0, 0.0), (0.0, 0.5, 0.0), (0.0, 0.0, 0.5),
        (0.0, 0.5, 0.5), (0.5, 0.0, 0.5), (0.5, 0.5, 0.0))


def yee_offsets():
    return _YEE


@dataclasses.dataclass(frozen=True)
class Config:
    name: str
    dim: int                      # 0 = uniform analytic field, 2 = 2D3V grid, 3 = 3D3V grid
    n_particles: int
    steps: int
    dt: float
    n_samples: int                # K frequency trials per particle and step
    hbar_n: float
    alpha: float = ALPHA
    grid: tuple = (1, 1, 1)       # cells (nx, ny, nz)
    dx: float = 1.0               # cell size (same on every axis)
    a0: float = 0.0               # per-beam amplitude of the standing wave
    b0: tuple = (0.0, 0.0, 0.0)   # uniform B for dim == 0
    recoil: int = 1               # 0 none, 1 photon, 2 Landau-Lifshitz
    kin_cut: bool = False
    photons_per_particle: int = 1  # photon-buffer capacity per particle and step
    seed: int = 0x5EED0001
    momentum: str = "thermal"     # "thermal" | "loguniform_gamma"
    temperature_mc2: float = 1.0 / 511.0
    gamma_range: tuple = (1.0, 1.0)  # log-uniform gamma range for "loguniform_gamma"
    slab: tuple | None = None     # (x_lo, x_hi) positions along x, or None for the full box
    sampler: int = 0              # 0 = S-proposal, 1 = table-direct, 2 = MLP-direct

    @property
    def box(self):
        return tuple(n * self.dx for n in self.grid)


_DX = TWO_PI / 64.0

CONFIGS = {
    # uniform 1e5 T field, omega_r = eB/m; dt = 0.01 gyro-periods at gamma = 1
    "c1": Config("c1_uniform_B_16k", 0, 16384, 1000, 0.01 * TWO_PI, 1, HBAR_N_1E5T,
                 b0=(0.0, 0.0, 1.0), momentum="loguniform_gamma", gamma_range=(10.0, 1e4),
                 photons_per_particle=1, seed=0x5EED0001),
    # 2048^2 2D3V, a0 = 300 standing wave, 1M electrons at 1 keV, 200 steps
    "c2": Config("c2_2d_2048sq_1M", 2, 1 << 20, 200, 0.5 * _DX, 1, HBAR_N_08UM,
                 grid=(2048, 2048, 1), dx=_DX, a0=300.0, photons_per_particle=4,
                 seed=0x5EED0002),
    # 512^3 3D3V, a0 = 500, 16M electrons in a 2-lambda slab, K = 8, 100 steps
    "c3": Config("c3_3d_512cube_16M_K8", 3, 1 << 24, 100, 0.5 * _DX, 8, HBAR_N_08UM,
                 grid=(512, 512, 512), dx=_DX, a0=500.0, kin_cut=True, photons_per_particle=8,
                 slab=(3 * TWO_PI, 5 * TWO_PI), seed=0x5EED0003),
    # the c3 workload driven through the learned (MLP) sampler
    "c4": Config("c4_3d_512cube_16M_K8_mlp", 3, 1 << 24, 100, 0.5 * _DX, 8, HBAR_N_08UM,
                 grid=(512, 512, 512), dx=_DX, a0=500.0, kin_cut=True, photons_per_particle=8,
                 slab=(3 * TWO_PI, 5 * TWO_PI), seed=0x5EED0004, sampler=2),
    # 768x768x384, a0 = 800, 64M electrons, gamma up to 3e4
    "c5": Config("c5_3d_768x768x384_64M", 3, 1 << 26, 20, 0.5 * _DX, 1, HBAR_N_08UM,
                 grid=(768, 768, 384), dx=_DX, a0=800.0, kin_cut=True, photons_per_particle=1,
                 momentum="loguniform_gamma", gamma_range=(1.0, 3e4), seed=0x5EED0005),
    # wakefield-shaped PIC-loop workload: 512x128x64 cells of lambda/32, an
    # underdense plasma (0.01 n_c, 2 electrons per cell, 1 keV) and a linearly
    # polarised laser pulse (a0 = 50) launched along x; the fields evolve
    # self-consistently (Yee solve, Esirkepov current)
    "c6": Config("c6_pic_wakefield_512x128x64", 3, 2 * 512 * 128 * 64, 40, 0.5 * TWO_PI / 32.0, 1,
                 HBAR_N_08UM, grid=(512, 128, 64), dx=TWO_PI / 32.0, a0=50.0, kin_cut=True,
                 photons_per_particle=1, seed=0x5EED0006),
}

# c6 plasma and pulse
C6_DENSITY = 0.01          # electron density in units of the critical density
C6_PULSE_X0 = 4.0 * TWO_PI  # pulse centre along x
C6_PULSE_SIGMA = 1.5 * TWO_PI   # rms length of the envelope
C6_PULSE_WAIST = 1.0 * TWO_PI   # transverse rms size


def config(name: str, **overrides) -> Config:
    return dataclasses.replace(CONFIGS[name], **overrides)


def _isotropic(rng, n):
    cos_t = rng.uniform(-1.0, 1.0, n)
    phi = rng.uniform(0.0, TWO_PI, n)
    sin_t = np.sqrt(np.maximum(0.0, 1.0 - cos_t * cos_t))
    return sin_t * np.cos(phi), sin_t * np.sin(phi), cos_t


def gen_particles(cfg: Config, n: int | None = None, seed: int | None = None,
                  dtype=np.float32) -> dict:
    """Initial macro-electron state (SoA): x, y, z, px, py, pz, w, id.

    Drawn in FP64 from numpy's PCG64 keyed by ``seed`` and rounded to ``dtype``.
    Positions are uniform over the box (or the slab); ids are 0..n-1; w = 1.
    """
    n = cfg.n_particles if n is None else int(n)
    rng = np.random.default_rng(cfg.seed if seed is None else seed)
    out = {}
    if cfg.dim == 0:
        x = y = z = np.zeros(n)
    else:
        L = cfg.box
        lo_x, hi_x = (0.0, L[0]) if cfg.slab is None else cfg.slab
        x = rng.uniform(lo_x, hi_x, n)
        y = rng.uniform(0.0, L[1], n)
        z = rng.uniform(0.0, L[2], n) if cfg.dim == 3 else np.zeros(n)
    if cfg.momentum == "thermal":
        s = math.sqrt(cfg.temperature_mc2)
        px, py, pz = rng.normal(0.0, s, n), rng.normal(0.0, s, n), rng.normal(0.0, s, n)
    else:
        g0, g1 = cfg.gamma_range
        gam = 10.0 ** rng.uniform(math.log10(g0), math.log10(g1), n)
        pm = np.sqrt(np.maximum(gam * gam - 1.0, 0.0))
        ux, uy, uz = _isotropic(rng, n)
        px, py, pz = pm * ux, pm * uy, pm * uz
    for k, v in (("x", x), ("y", y), ("z", z), ("px", px), ("py", py), ("pz", pz)):
        out[k] = np.ascontiguousarray(v, dtype=dtype)
    if cfg.dim != 0:
        # keep rounded positions inside [0, L)
        for k, a in (("x", 0), ("y", 1), ("z", 2)):
            L = cfg.box[a]
            v = out[k]
            v[v >= dtype(L)] = dtype(0.0)
    out["w"] = np.ones(n, dtype=dtype)
    out["id"] = np.arange(n, dtype=np.uint32)
    return out


def field_at(cfg: Config, x, t: float):
    """Standing wave of two counter-propagating circularly polarised beams of
    amplitude a0 along x (k = omega = 1):
        E = 2 a0 cos x (0,  cos t, -sin t),   B = 2 a0 sin x (0, -cos t, sin t).
    Returns (E, B) as lists of three arrays evaluated at x (FP64)."""
    x = np.asarray(x, dtype=np.float64)
    a = 2.0 * cfg.a0
    cx, sx = np.cos(x), np.sin(x)
    ct, st = math.cos(t), math.sin(t)
    z = np.zeros_like(x)
    E = [z, a * cx * ct, -a * cx * st]
    B = [z, -a * sx * ct, a * sx * st]
    return E, B


def standing_wave_grid(cfg: Config, t: float, dtype=np.float32):
    """The standing wave sampled at the Yee points of the grid at time t.

    Returns (E, B): two lists of three flat arrays of nx*ny*nz values, x fastest.
    Each component depends on x only, so it is built from a 1D profile."""
    nx, ny, nz = cfg.grid
    if cfg.dim == 2:
        nz = 1
    E_out, B_out = [], []
    for c in range(6):
        xs = (np.arange(nx, dtype=np.float64) + _YEE[c][0]) * cfg.dx
        E, B = field_at(cfg, xs, t)
        prof = (E + B)[c].astype(dtype)
        arr = np.empty((nz, ny, nx), dtype=dtype)
        arr[...] = prof[None, None, :]
        (E_out if c < 3 else B_out).append(arr.reshape(-1))
    return E_out, B_out


def plasma_weight(cfg: Config, density: float) -> float:
    """Weight of each of cfg.n_particles electrons spread uniformly over the box
    so that they make `density` (in units of n_r, (c/omega_r)^-3)."""
    vol = 1.0
    for L in cfg.box[:cfg.dim]:
        vol *= L
    return density * vol / cfg.n_particles


def laser_pulse_grid(cfg: Config, t: float = 0.0, dtype=np.float32):
    """A linearly polarised (E along y) pulse moving along +x in vacuum form,
    sampled at the Yee points: Ey = a0 cos(x - t) g, Bz = Ey (at its own
    points), g a Gaussian envelope centred at C6_PULSE_X0 + t (rms length
    C6_PULSE_SIGMA) times a transverse Gaussian of rms size C6_PULSE_WAIST about
    the box axis.  Returns (E, B) as flat arrays, x fastest."""
    nx, ny, nz = cfg.grid
    L = cfg.box
    out = []
    for c in range(6):
        off = _YEE[c]
        x = (np.arange(nx, dtype=np.float64) + off[0]) * cfg.dx
        y = (np.arange(ny, dtype=np.float64) + off[1]) * cfg.dx - 0.5 * L[1]
        z = (np.arange(nz, dtype=np.float64) + off[2]) * cfg.dx - 0.5 * L[2]
        if c not in (1, 5):
            out.append(np.zeros(nx * ny * nz, dtype=dtype))
            continue
        phase = x - t
        gx = cfg.a0 * np.cos(phase) * np.exp(-0.5 * ((x - C6_PULSE_X0 - t) / C6_PULSE_SIGMA) ** 2)
        gy = np.exp(-0.5 * (y / C6_PULSE_WAIST) ** 2)
        gz = np.exp(-0.5 * (z / C6_PULSE_WAIST) ** 2)
        arr = gz[:, None, None] * gy[None, :, None] * gx[None, None, :]
        out.append(arr.astype(dtype).reshape(-1))
    return out[:3], out[3:]

