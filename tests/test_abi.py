"""C-ABI checks that need no GPU: the library loads, exports every function
include/sr.h declares, and rejects bad arguments on the host (no launch)."""
import ctypes as C
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "sr.h")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = set(re.findall(r"\b(sr_[a-z0-9_]+)\s*\(", text))
    return sorted(names)


@pytest.fixture(scope="module")
def lib():
    from paper_1409_5574_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        from paper_1409_5574_amd import build
        build.build()
    return _lib.load()


def test_header_declares_entry_points():
    names = _declared()
    for must in ("sr_gather_push_emit", "sr_gather_push_emit_f64", "sr_energy_ledger",
                 "sr_table_build", "sr_table_free", "sr_status", "sr_strerror"):
        assert must in names


def test_boundary_calls_of_the_hot_path():
    # the calls the path's boundary is specified with: the step (FP32 and FP64),
    # the ledger, the tables, the surrogate's forward, backward and Adam step,
    # the status word and error text
    names = _declared()
    for must in ("sr_gather_push_emit", "sr_gather_push_emit_f64", "sr_energy_ledger",
                 "sr_table_build", "sr_table_free", "sr_mlp_forward", "sr_mlp_backward",
                 "sr_mlp_adam", "sr_status", "sr_strerror"):
        assert must in names, must


def test_library_exports_every_declared_symbol(lib):
    from paper_1409_5574_amd import _lib
    out = subprocess.run(["nm", "-D", "--defined-only", _lib.LIB_PATH], capture_output=True,
                         text=True, check=True).stdout
    exported = {line.split()[-1] for line in out.splitlines() if line.strip()}
    missing = [n for n in _declared() if n not in exported]
    assert not missing, missing
    # and the Python binding knows every one of them
    assert set(_declared()) <= set(_lib.SIGNATURES)


def test_strerror_and_sizes(lib):
    from paper_1409_5574_amd import _lib as L
    assert lib.sr_strerror(0) == b"ok"
    assert lib.sr_strerror(L.SR_E_INVAL) == b"invalid argument"
    assert lib.sr_strerror(12345) == b"unknown error code"
    assert lib.sr_ledger_partials(100) >= 100 * L.SR_LEDGER_COLS
    assert lib.sr_ledger_partials(-1) == 0
    assert lib.sr_hist_work(64) > 0 and lib.sr_hist_work(0) == -1 and lib.sr_hist_work(5000) == -1
    assert lib.sr_angular_work(45, 72) > 45 * 72
    assert lib.sr_angular_work(0, 8) == -1 and lib.sr_angular_work(65, 64) == -1
    g = L.Grid()
    g.dim = 3
    for a in range(3):
        g.n[a] = 64
        g.dx[a] = 0.1
    tile = (C.c_int32 * 3)(8, 8, 8)
    assert lib.sr_sort_work(C.byref(g), tile, 1000) > 4 * 1000
    bad = (C.c_int32 * 3)(0, 8, 8)
    assert lib.sr_sort_work(C.byref(g), bad, 1000) == -1


def test_step_rejects_bad_arguments_on_host(lib):
    from paper_1409_5574_amd import _lib as L
    p = L.Particles32()
    p.n = 10
    grid = L.Grid()
    grid.dim = 0
    prm = L.Params(1e-5, 7.3e-3, 1, 0, 1, 0, 0, 0)
    ch = L.Chunking(1, None)
    ph = L.PhotonBuf()
    led = L.Ledger()
    args = dict(dt=0.1, seed=1, step=0)
    # null particle arrays with n > 0
    rc = lib.sr_gather_push_emit(C.byref(p), None, C.byref(grid), args["dt"], 1, 0, C.byref(prm),
                                 None, C.byref(ch), C.byref(ph), C.byref(led), None)
    assert rc == L.SR_E_INVAL
    # bad K, bad dt, bad grid dim: all caught before any launch
    dummy = C.c_void_p(16)
    for a in range(3):
        p.p[a] = dummy
    p.w = dummy
    p.id = dummy
    for bad_prm, dt, dim in ((L.Params(1e-5, 7.3e-3, 0, 0, 1, 0, 0, 0), 0.1, 0),
                             (prm, -1.0, 0), (prm, 0.1, 1),
                             (L.Params(1e-5, 7.3e-3, 17, 0, 1, 0, 0, 0), 0.1, 0),
                             (L.Params(0.0, 7.3e-3, 1, 0, 1, 0, 0, 0), 0.1, 0)):
        grid.dim = dim
        rc = lib.sr_gather_push_emit(C.byref(p), None, C.byref(grid), dt, 1, 0, C.byref(bad_prm),
                                     dummy, C.byref(ch), C.byref(ph), C.byref(led), None)
        assert rc == L.SR_E_INVAL
    # an unknown gather mode
    grid.dim = 0
    bad_gather = L.Params(1e-5, 7.3e-3, 1, 0, 1, 0, 0, 0, None, None, 0.0, 2)
    assert lib.sr_gather_push_emit(C.byref(p), None, C.byref(grid), 0.1, 1, 0, C.byref(bad_gather),
                                   dummy, C.byref(ch), C.byref(ph), C.byref(led),
                                   None) == L.SR_E_INVAL
    # multi-step launches: uniform fields, no learned sampler, no grid floor
    g3 = L.Grid()
    g3.dim = 3
    assert lib.sr_gather_push_emit_steps(C.byref(p), C.byref(g3), 0.1, 1, 0, 10, C.byref(prm),
                                         dummy, C.byref(ph), C.byref(led),
                                         None) == L.SR_E_UNSUPPORTED
    mlp_prm = L.Params(1e-5, 7.3e-3, 1, 2, 1, 0, 0, 0, dummy, dummy)
    assert lib.sr_gather_push_emit_steps(C.byref(p), C.byref(grid), 0.1, 1, 0, 10, C.byref(mlp_prm),
                                         dummy, C.byref(ph), C.byref(led),
                                         None) == L.SR_E_UNSUPPORTED
    assert lib.sr_gather_push_emit_steps(C.byref(p), C.byref(grid), 0.1, 1, 0, 0, C.byref(prm),
                                         dummy, C.byref(ph), C.byref(led), None) == L.SR_E_INVAL
    assert lib.sr_table_build(None, None) == L.SR_E_INVAL
    assert lib.sr_energy_ledger(None, 0, None, None) == L.SR_E_INVAL
    assert lib.sr_ledger_reduce(None, 1, 0, None) == L.SR_E_INVAL
    assert lib.sr_ledger_reduce(C.byref(led), 1, 0, None) == L.SR_E_INVAL


def test_eval_push_rejects_bad_arguments_on_host(lib):
    from paper_1409_5574_amd import _lib as L
    p = L.Particles32()
    p.n = 10
    grid = L.Grid()
    grid.dim = 0
    prm = L.Params(1e-5, 7.3e-3, 1, 0, 1, 0, 0, 0)
    out = C.c_void_p(16)
    # null particle arrays with n > 0
    assert lib.sr_eval_push(C.byref(p), None, C.byref(grid), 0.1, C.byref(prm), out, out, out,
                            None) == L.SR_E_INVAL
    dummy = C.c_void_p(16)
    for a in range(3):
        p.p[a] = dummy
    p.w = dummy
    p.id = dummy
    # null outputs, bad dt, bad hbar_n, a 2D grid without fields or with nx < 2
    assert lib.sr_eval_push(C.byref(p), None, C.byref(grid), 0.1, C.byref(prm), None, out, out,
                            None) == L.SR_E_INVAL
    assert lib.sr_eval_push(C.byref(p), None, C.byref(grid), 0.0, C.byref(prm), out, out, out,
                            None) == L.SR_E_INVAL
    bad = L.Params(0.0, 7.3e-3, 1, 0, 1, 0, 0, 0)
    assert lib.sr_eval_push(C.byref(p), None, C.byref(grid), 0.1, C.byref(bad), out, out, out,
                            None) == L.SR_E_INVAL
    grid.dim = 2
    grid.n[0], grid.n[1], grid.n[2] = 1, 8, 1
    grid.dx[0] = grid.dx[1] = grid.dx[2] = 0.1
    assert lib.sr_eval_push(C.byref(p), None, C.byref(grid), 0.1, C.byref(prm), out, out, out,
                            None) == L.SR_E_INVAL
    f = L.Fields32()
    for a in range(3):
        f.e[a] = dummy
        f.b[a] = dummy
    p.x[0] = p.x[1] = dummy
    assert lib.sr_eval_push(C.byref(p), C.byref(f), C.byref(grid), 0.1, C.byref(prm), out, out,
                            out, None) == L.SR_E_INVAL
    # an empty set is a no-op
    p.n = 0
    grid.dim = 0
    assert lib.sr_eval_push(C.byref(p), None, C.byref(grid), 0.1, C.byref(prm), None, None, None,
                            None) == L.SR_OK


def test_angular_histogram_rejects_bad_arguments_on_host(lib):
    from paper_1409_5574_amd import _lib as L
    ph = L.PhotonBuf()
    ch = L.Chunking(1, None)
    out = C.c_void_p(16)
    ax = (C.c_double * 3)(1.0, 0.0, 0.0)
    rf = (C.c_double * 3)(0.0, 1.0, 0.0)
    # null photon buffer, no segment counts
    assert lib.sr_angular_histogram(None, C.byref(ch), 10, ax, rf, 8, 8, out, out, None) == L.SR_E_INVAL
    assert lib.sr_angular_histogram(C.byref(ph), C.byref(ch), 10, ax, rf, 8, 8, out, out,
                                    None) == L.SR_E_INVAL
    ph.seg_count = out
    # zero axis, reference parallel to the axis, bad bin counts: caught before a launch
    zero = (C.c_double * 3)(0.0, 0.0, 0.0)
    par = (C.c_double * 3)(-3.0, 0.0, 0.0)
    for a, r, nt, nph in ((zero, rf, 8, 8), (ax, par, 8, 8), (ax, zero, 8, 8), (ax, rf, 0, 8),
                          (ax, rf, 8, -1), (ax, rf, 4096, 2)):
        assert lib.sr_angular_histogram(C.byref(ph), C.byref(ch), 10, a, r, nt, nph, out, out,
                                        None) == L.SR_E_INVAL


def test_eval_trial_quantum_rejects_bad_arguments_on_host(lib):
    from paper_1409_5574_amd import _lib as L
    d = C.c_void_p(16)
    assert lib.sr_eval_trial_quantum(None, d, d, d, d, d, 4, None) == L.SR_E_INVAL
    assert lib.sr_eval_trial_quantum(d, None, d, d, d, d, 4, None) == L.SR_E_INVAL
    assert lib.sr_eval_trial_quantum(d, d, d, d, d, d, -1, None) == L.SR_E_INVAL
    assert lib.sr_eval_trial_quantum(d, None, None, None, None, None, 0, None) == L.SR_OK


def test_validity_and_floor_reject_bad_arguments_on_host(lib):
    from paper_1409_5574_amd import _lib as L
    p = L.Particles32()
    p.n = 10
    d = C.c_void_p(16)
    for a in range(3):
        p.p[a] = d
    p.w = d
    p.id = d
    grid = L.Grid()
    grid.dim = 0
    prm = L.Params(1e-5, 7.3e-3, 1, 0, 1, 0, 0, 0, None, None, 0.0)
    assert lib.sr_validity_work(1000) >= 6 and lib.sr_validity_work(-1) == -1
    # tau_em must be positive; sums and work are required
    assert lib.sr_validity(C.byref(p), None, C.byref(grid), 0.1, C.byref(prm), 0.0, None, d, d,
                           None) == L.SR_E_INVAL
    assert lib.sr_validity(C.byref(p), None, C.byref(grid), 0.1, C.byref(prm), 1.0, None, None, d,
                           None) == L.SR_E_INVAL
    ch = L.Chunking(1, None)
    ph = L.PhotonBuf()
    led = L.Ledger()
    # a negative grid frequency, and the floor with the learned sampler
    for bad in (L.Params(1e-5, 7.3e-3, 1, 0, 1, 0, 0, 0, None, None, -1.0),
                L.Params(1e-5, 7.3e-3, 1, 2, 1, 0, 0, 0, d, d, 5.0)):
        rc = lib.sr_gather_push_emit(C.byref(p), None, C.byref(grid), 0.1, 1, 0, C.byref(bad), d,
                                     C.byref(ch), C.byref(ph), C.byref(led), None)
        assert rc == L.SR_E_INVAL


def test_pic_calls_reject_bad_arguments_on_host(lib):
    from paper_1409_5574_amd import _lib as L
    d = C.c_void_p(16)
    g = L.Grid()
    g.dim = 3
    for a in range(3):
        g.n[a] = 8
        g.dx[a] = 0.1
    e = L.P3(d, d, d)
    b = L.P3(d, d, d)
    none = L.P3(None, None, None)
    # the Courant condition dt^2 sum 1/dx^2 < 1: 0.1/sqrt(3) = 0.0577
    assert lib.sr_field_step(e, b, none, C.byref(g), 0.06, None) == L.SR_E_INVAL
    assert lib.sr_field_step(e, b, none, C.byref(g), 0.0, None) == L.SR_E_INVAL
    assert lib.sr_field_step(L.P3(d, None, d), b, none, C.byref(g), 0.05, None) == L.SR_E_INVAL
    # a current with a missing component
    assert lib.sr_field_step(e, b, L.P3(d, None, d), C.byref(g), 0.05, None) == L.SR_E_INVAL
    g0 = L.Grid()
    g0.dim = 0
    assert lib.sr_field_step(e, b, none, C.byref(g0), 0.05, None) == L.SR_E_INVAL
    p = L.Particles32()
    p.n = 10
    for a in range(3):
        p.x[a] = d
        p.p[a] = d
    p.w = d
    p.id = d
    j = L.P3(d, d, d)
    xo = L.P3(d, d, d)
    # status, current and old positions are required; dt > 0
    assert lib.sr_deposit_current(C.byref(p), xo, C.byref(g), 0.05, -1.0, j, None, None) == L.SR_E_INVAL
    assert lib.sr_deposit_current(C.byref(p), xo, C.byref(g), 0.05, -1.0, L.P3(d, None, d), d,
                                  None) == L.SR_E_INVAL
    assert lib.sr_deposit_current(C.byref(p), L.P3(d, None, d), C.byref(g), 0.05, -1.0, j, d,
                                  None) == L.SR_E_INVAL
    assert lib.sr_deposit_current(C.byref(p), xo, C.byref(g), 0.0, -1.0, j, d, None) == L.SR_E_INVAL
    assert lib.sr_deposit_rho(C.byref(p), C.byref(g0), -1.0, d, None) == L.SR_E_INVAL
    assert lib.sr_deposit_rho(C.byref(p), C.byref(g), -1.0, None, None) == L.SR_E_INVAL
    ph = L.PhotonBuf()
    ch = L.Chunking(1, None)
    assert lib.sr_photon_advance(C.byref(ph), C.byref(ch), 10, C.byref(g), 0.05, None) == L.SR_E_INVAL
    ph.seg_count = d
    assert lib.sr_photon_advance(C.byref(ph), C.byref(ch), 10, C.byref(g), -1.0, None) == L.SR_E_INVAL
    # the multi-step launch is for uniform fields only
    assert lib.sr_gather_push_emit_steps(C.byref(p), C.byref(g), 0.05, 1, 0, 10, None, None, None,
                                         None, None) == L.SR_E_INVAL
    # sizes whose byte offsets would not fit the kernels' 32-bit offsets
    p.n = 1 << 29
    assert lib.sr_deposit_rho(C.byref(p), C.byref(g), -1.0, d, None) == L.SR_E_UNSUPPORTED
    assert lib.sr_deposit_current(C.byref(p), xo, C.byref(g), 0.05, -1.0, j, d,
                                  None) == L.SR_E_UNSUPPORTED
    ph.per_particle = 4
    ph.dir[0] = ph.dir[1] = ph.dir[2] = d
    ch = L.Chunking(1 << 23, None)
    assert lib.sr_photon_advance(C.byref(ph), C.byref(ch), 1 << 28, C.byref(g), 0.05,
                                 None) == L.SR_E_UNSUPPORTED


def test_step_epilogue_rejects_bad_arguments_on_host(lib):
    """The epilogue takes the checks of both calls it fuses, before any launch."""
    from paper_1409_5574_amd import _lib as L
    d = C.c_void_p(16)
    led = L.Ledger()
    led.rows, led.partials, led.status = d, d, d
    led.n_rows = 2
    led.partials_len = lib.sr_ledger_partials(8)
    ph = L.PhotonBuf()
    ph.seg_count = d
    ch = L.Chunking(8, None)

    def call(ledger=C.byref(led), n_chunks=8, row=0, photons=C.byref(ph), chunks=C.byref(ch),
             n=500, lo=1e-6, hi=1e4, bins=16, hist=d, work=d):
        return lib.sr_step_epilogue(ledger, n_chunks, row, photons, chunks, n, lo, hi, bins, hist,
                                    work, None)

    assert call(ledger=None) == L.SR_E_INVAL
    assert call(row=2) == L.SR_E_INVAL                 # past the ledger's rows
    assert call(n_chunks=-1) == L.SR_E_INVAL
    assert call(n_chunks=1 << 20) == L.SR_E_INVAL      # partials too short
    assert call(photons=None) == L.SR_E_INVAL
    assert call(chunks=None) == L.SR_E_INVAL
    assert call(hist=None) == L.SR_E_INVAL
    assert call(work=None) == L.SR_E_INVAL
    assert call(bins=0) == L.SR_E_INVAL
    assert call(bins=1025) == L.SR_E_INVAL
    assert call(lo=0.0) == L.SR_E_INVAL
    assert call(hi=1e-7) == L.SR_E_INVAL                # hi below lo
    ph.per_particle = 2                                 # slots but no eps / w arrays
    assert call() == L.SR_E_INVAL
