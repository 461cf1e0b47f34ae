"""Closing the PIC loop around the emission step: the Yee field solve and the
grid charge/current, in plain FP64 (test infrastructure only; imports nothing
from the HIP package).

The emission method of the paper runs inside a PIC code: particles on a grid,
Maxwell's equations for the field, the particles' currents feeding the field
(section "The field setup").  Normalised units: E, B in m c omega_r / e,
lengths in c/omega_r, time in 1/omega_r, densities in n_r = m omega_r^2 /
(4 pi e^2), so that

    dB/dt = -curl E,    dE/dt = curl B - J,    div E = rho.

Yee lattice, component-major arrays of shape (nz, ny, nx) (x fastest; 2D has
nz = 1 and no z dependence), periodic:
    Ex (i+1/2, j, k)   Ey (i, j+1/2, k)   Ez (i, j, k+1/2)
    Bx (i, j+1/2, k+1/2)   By (i+1/2, j, k+1/2)   Bz (i+1/2, j+1/2, k)
    Jx, Jy, Jz on the E points; rho on the nodes (i, j, k).
One step keeps E and B at whole steps (the particles gather both at t^n):
    B <- B - (dt/2) curl E;  E <- E + dt (curl B - J);  B <- B - (dt/2) curl E.
"""
from __future__ import annotations

import ctypes as C

import numpy as np

from . import oracle as _o


def _fwd(a, axis, d):
    """(a[i+1] - a[i]) / d along axis (periodic); axis 0 = z, 1 = y, 2 = x."""
    return (np.roll(a, -1, axis=axis) - a) / d


def _bwd(a, axis, d):
    """(a[i] - a[i-1]) / d along axis (periodic)."""
    return (a - np.roll(a, 1, axis=axis)) / d


def curl_E(E, dx):
    """curl E on the B points: forward differences."""
    Ex, Ey, Ez = E
    ddx, ddy, ddz = dx
    return (_fwd(Ez, 1, ddy) - _fwd(Ey, 0, ddz),
            _fwd(Ex, 0, ddz) - _fwd(Ez, 2, ddx),
            _fwd(Ey, 2, ddx) - _fwd(Ex, 1, ddy))


def curl_B(B, dx):
    """curl B on the E points: backward differences."""
    Bx, By, Bz = B
    ddx, ddy, ddz = dx
    return (_bwd(Bz, 1, ddy) - _bwd(By, 0, ddz),
            _bwd(Bx, 0, ddz) - _bwd(Bz, 2, ddx),
            _bwd(By, 2, ddx) - _bwd(Bx, 1, ddy))


def div_E(E, dx):
    """div E on the nodes (backward differences of the staggered components)."""
    return _bwd(E[0], 2, dx[0]) + _bwd(E[1], 1, dx[1]) + _bwd(E[2], 0, dx[2])


def div_B(B, dx):
    """div B on the cell centres (forward differences)."""
    return _fwd(B[0], 2, dx[0]) + _fwd(B[1], 1, dx[1]) + _fwd(B[2], 0, dx[2])


def fdtd_step(E, B, J, dt, dx):
    """One step of the Yee scheme with B split around the E update (in place on
    lists of arrays).  J: the current of the step (t^{n+1/2}), or None."""
    c = curl_E(E, dx)
    for q in range(3):
        B[q] -= 0.5 * dt * c[q]
    c = curl_B(B, dx)
    for q in range(3):
        E[q] += dt * (c[q] - (0.0 if J is None else J[q]))
    c = curl_E(E, dx)
    for q in range(3):
        B[q] -= 0.5 * dt * c[q]


def _lib():
    L = _o.lib()
    if not getattr(L, "_pic_bound", False):
        p, d, i64, i32 = C.c_void_p, C.c_double, C.c_int64, C.c_int32
        L.orc_deposit_rho.restype = C.c_int
        L.orc_deposit_rho.argtypes = [i64, p, p, p, p, d, i32, p, p, p]
        L.orc_deposit_current.restype = C.c_int
        L.orc_deposit_current.argtypes = [i64, p, p, p, p, p, p, p, p, d, d, i32, p, p, p, p, p]
        L._pic_bound = True
    return L


def _arr(a):
    return None if a is None else np.ascontiguousarray(a, dtype=np.float64)


def deposit_rho(pos, w, q, dim, n, dx):
    """CIC charge density on the nodes, shape (nz, ny, nx); pos: (N, dim)."""
    pos = np.asarray(pos, np.float64)
    x, y = _arr(pos[:, 0]), _arr(pos[:, 1])
    z = _arr(pos[:, 2]) if dim == 3 else None
    w = _arr(w)
    nz = n[2] if dim == 3 else 1
    rho = np.zeros((nz, n[1], n[0]))
    nn = (C.c_int64 * 3)(*[int(v) for v in n])
    dd = (C.c_double * 3)(*[float(v) for v in dx])
    rc = _lib().orc_deposit_rho(x.size, _o._ptr(x), _o._ptr(y), _o._ptr(z), _o._ptr(w), float(q),
                                int(dim), nn, dd, _o._ptr(rho))
    if rc != 0:
        raise RuntimeError(f"orc_deposit_rho failed ({rc})")
    return rho


def deposit_current(pos0, pos1, vz, w, q, dt, dim, n, dx):
    """Esirkepov current of the moves pos0 -> pos1: (Jx, Jy, Jz), each (nz, ny, nx)."""
    pos0 = np.asarray(pos0, np.float64)
    pos1 = np.asarray(pos1, np.float64)
    cols = [_arr(pos0[:, a]) if a < dim else None for a in range(3)]
    cols1 = [_arr(pos1[:, a]) if a < dim else None for a in range(3)]
    vz = _arr(vz) if dim == 2 else None
    w = _arr(w)
    nz = n[2] if dim == 3 else 1
    J = [np.zeros((nz, n[1], n[0])) for _ in range(3)]
    nn = (C.c_int64 * 3)(*[int(v) for v in n])
    dd = (C.c_double * 3)(*[float(v) for v in dx])
    rc = _lib().orc_deposit_current(w.size, *[_o._ptr(c) for c in cols], *[_o._ptr(c) for c in cols1],
                                    _o._ptr(vz), _o._ptr(w), float(q), float(dt), int(dim), nn, dd,
                                    *[_o._ptr(j) for j in J])
    if rc != 0:
        raise RuntimeError(f"orc_deposit_current failed ({rc})")
    return J


def photon_advance(pos, direction, dt, box):
    """Photons move at c along their direction (periodic box); pos (N, 3)."""
    out = np.asarray(pos, np.float64) + dt * np.asarray(direction, np.float64)
    for a, L in enumerate(box):
        if L is not None:
            out[:, a] = np.mod(out[:, a], L)
    return out
