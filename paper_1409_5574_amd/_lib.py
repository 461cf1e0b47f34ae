"""ctypes mirror of include/sr.h and the loader of libsr.so.

Argument marshalling only: every step of the emission path runs in the HIP
kernels of libsr.so.  If the library is missing, loading raises -- there is no
CPU fallback.
"""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libsr.so")

SR_OK, SR_E_INVAL, SR_E_HIP, SR_E_NOMEM, SR_E_UNSUPPORTED = 0, -1, -2, -3, -4
SR_W_PHOTON_OVERFLOW, SR_W_RECOIL_CLAMP, SR_W_NONFINITE, SR_W_CFL = 1, 2, 4, 8
(SR_LED_EMITTED, SR_LED_LL, SR_LED_RECOIL, SR_LED_CLAMPED, SR_LED_DROPPED, SR_LED_PHOTONS,
 SR_LED_WEIGHT, SR_LED_CHI_MAX) = range(8)
SR_LEDGER_COLS = 8
SR_CHUNK = 64
SR_NOALLOC_MAX_CHUNKS = 1 << 20
SR_SAMPLER_S, SR_SAMPLER_TABLE, SR_SAMPLER_MLP, SR_SAMPLER_QUANTUM = 0, 1, 2, 3
SR_RECOIL_NONE, SR_RECOIL_PHOTON, SR_RECOIL_LL = 0, 1, 2
SR_DN_WEIGHT, SR_DN_CLAMP = 0, 1
SR_GATHER_DIRECT, SR_GATHER_BOX = 0, 1
SR_FIELD_BOX_NODES = 1344
SR_VALID_QUANTUM, SR_VALID_NON_SYNCHROTRON, SR_VALID_SUMS = 1, 2, 6
SR_MLP_PARAMS = 8577
SR_MLP_FALLBACK_BINS = 24

P3 = C.c_void_p * 3


class Particles32(C.Structure):
    _fields_ = [("n", C.c_int64), ("x", P3), ("p", P3), ("w", C.c_void_p), ("id", C.c_void_p)]


class Particles64(C.Structure):
    _fields_ = [("n", C.c_int64), ("x", P3), ("p", P3), ("w", C.c_void_p), ("id", C.c_void_p)]


class Fields32(C.Structure):
    _fields_ = [("e", P3), ("b", P3)]


class Grid(C.Structure):
    _fields_ = [("dim", C.c_int32), ("reserved", C.c_int32), ("n", C.c_int64 * 3),
                ("dx", C.c_double * 3), ("e0", C.c_double * 3), ("b0", C.c_double * 3)]


class Params(C.Structure):
    _fields_ = [("hbar_n", C.c_double), ("alpha", C.c_double), ("n_samples", C.c_int32),
                ("sampler", C.c_int32), ("recoil", C.c_int32), ("dn_policy", C.c_int32),
                ("kin_cut", C.c_int32), ("push_position", C.c_int32),
                ("mlp_params", C.c_void_p), ("mlp_fallback", C.c_void_p),
                ("omega_grid", C.c_double), ("gather", C.c_int32), ("reserved", C.c_int32)]


class Chunking(C.Structure):
    _fields_ = [("n_chunks", C.c_int64), ("start", C.c_void_p)]


class PhotonBuf(C.Structure):
    _fields_ = [("per_particle", C.c_int64), ("seg_count", C.c_void_p), ("eps", C.c_void_p),
                ("w", C.c_void_p), ("dir", P3), ("pos", P3), ("parent", C.c_void_p),
                ("k", C.c_void_p), ("step", C.c_void_p)]


class Ledger(C.Structure):
    _fields_ = [("rows", C.c_void_p), ("n_rows", C.c_int64), ("partials", C.c_void_p),
                ("partials_len", C.c_int64), ("status", C.c_void_p)]


class TableInfo(C.Structure):
    _fields_ = [("proposal_pa", C.c_float), ("f_pieces", C.c_int32), ("proposal_a", C.c_double),
                ("t1_pieces", C.c_int32), ("r_nodes", C.c_int32), ("r_log10chi_lo", C.c_double),
                ("r_log10chi_hi", C.c_double), ("g_pieces", C.c_int32),
                ("q_pieces", C.c_int32)]


# name -> (restype, argtypes); every symbol include/sr.h declares
_P, _I64, _I32, _U64, _D = C.c_void_p, C.c_int64, C.c_int32, C.c_uint64, C.c_double
SIGNATURES = {
    "sr_table_build": (C.c_int, [C.POINTER(C.c_void_p), _P]),
    "sr_table_free": (None, [_P]),
    "sr_table_query": (C.c_int, [_P, C.POINTER(TableInfo)]),
    "sr_eval_synchrotron_F": (C.c_int, [_P, _P, _P, _I64, _P]),
    "sr_eval_trial": (C.c_int, [_P, _P, _P, _P, _I32, _P, _P, _I64, _P]),
    "sr_eval_trial_quantum": (C.c_int, [_P, _P, _P, _P, _P, _P, _I64, _P]),
    "sr_validity": (C.c_int, [C.POINTER(Particles32), C.POINTER(Fields32), C.POINTER(Grid),
                              C.c_double, C.POINTER(Params), C.c_double, _P, _P, _P, _P]),
    "sr_validity_work": (C.c_int64, [_I64]),
    "sr_field_step": (C.c_int, [P3, P3, P3, C.POINTER(Grid), _D, _P]),
    "sr_deposit_rho": (C.c_int, [C.POINTER(Particles32), C.POINTER(Grid), _D, _P, _P]),
    "sr_deposit_current": (C.c_int, [C.POINTER(Particles32), P3, C.POINTER(Grid), _D, _D, P3, _P,
                                     _P]),
    "sr_photon_advance": (C.c_int, [C.POINTER(PhotonBuf), C.POINTER(Chunking), _I64,
                                    C.POINTER(Grid), _D, _P]),
    "sr_philox": (C.c_int, [_P, _U64, _P, _I64, _P]),
    "sr_gather_push_emit": (C.c_int, [C.POINTER(Particles32), C.POINTER(Fields32),
                                      C.POINTER(Grid), _D, _U64, _U64, C.POINTER(Params), _P,
                                      C.POINTER(Chunking), C.POINTER(PhotonBuf),
                                      C.POINTER(Ledger), _P]),
    "sr_gather_push_emit_timed": (C.c_int, [C.POINTER(Particles32), C.POINTER(Fields32),
                                            C.POINTER(Grid), _D, _U64, _U64, C.POINTER(Params),
                                            _P, C.POINTER(Chunking), C.POINTER(PhotonBuf),
                                            C.POINTER(Ledger), _P, _P, _P]),
    "sr_gather_push_emit_f64": (C.c_int, [C.POINTER(Particles64), C.POINTER(Fields32),
                                          C.POINTER(Grid), _D, _U64, _U64, C.POINTER(Params), _P,
                                          C.POINTER(Chunking), C.POINTER(PhotonBuf),
                                          C.POINTER(Ledger), _P]),
    "sr_eval_push": (C.c_int, [C.POINTER(Particles32), C.POINTER(Fields32), C.POINTER(Grid), _D,
                               C.POINTER(Params), _P, _P, _P, _P]),
    "sr_eval_push_f64": (C.c_int, [C.POINTER(Particles64), C.POINTER(Fields32), C.POINTER(Grid),
                                   _D, C.POINTER(Params), _P, _P, _P, _P]),
    "sr_gather_push_emit_noalloc": (C.c_int, [C.POINTER(Particles32), C.POINTER(Fields32),
                                              C.POINTER(Grid), _D, _U64, _U64,
                                              C.POINTER(Params), _P, C.POINTER(Chunking),
                                              C.POINTER(PhotonBuf), _P, _P, _P]),
    "sr_gather_push_emit_steps": (C.c_int, [C.POINTER(Particles32), C.POINTER(Grid), _D, _U64,
                                            _U64, _I64, C.POINTER(Params), _P,
                                            C.POINTER(PhotonBuf), C.POINTER(Ledger), _P]),
    "sr_ledger_partials_steps": (C.c_int64, [_I64, _I64]),
    "sr_ledger_reduce": (C.c_int, [C.POINTER(Ledger), _I64, _I64, _P]),
    "sr_ledger_partials": (C.c_int64, [_I64]),
    "sr_energy_ledger": (C.c_int, [C.POINTER(Ledger), _I64, _P, _P]),
    "sr_status": (C.c_int, [C.POINTER(Ledger), C.POINTER(C.c_uint32), _I32, _P]),
    "sr_spectrum_histogram": (C.c_int, [C.POINTER(PhotonBuf), C.POINTER(Chunking), _I64, _D, _D,
                                        _I32, _P, _P, _P]),
    "sr_step_epilogue": (C.c_int, [C.POINTER(Ledger), _I64, _I64, C.POINTER(PhotonBuf),
                                   C.POINTER(Chunking), _I64, _D, _D, _I32, _P, _P, _P]),
    "sr_hist_work": (C.c_int64, [_I32]),
    "sr_angular_histogram": (C.c_int, [C.POINTER(PhotonBuf), C.POINTER(Chunking), _I64,
                                       C.POINTER(C.c_double), C.POINTER(C.c_double), _I32, _I32,
                                       _P, _P, _P]),
    "sr_angular_work": (C.c_int64, [_I32, _I32]),
    "sr_field_standing_wave": (C.c_int, [P3, P3, C.POINTER(Grid), _D, _D, _P]),
    "sr_sort_particles": (C.c_int, [C.POINTER(Particles32), C.POINTER(Particles32),
                                    C.POINTER(Grid), C.POINTER(C.c_int32), _P, _P]),
    "sr_sort_work": (C.c_int64, [C.POINTER(Grid), C.POINTER(C.c_int32), _I64]),
    "sr_strerror": (C.c_char_p, [C.c_int]),
    "sr_mlp_forward": (C.c_int, [_P, _P, _P, _I64, _P]),
    "sr_mlp_mse_grad": (C.c_int, [_P, _P, _P, _I64, _P, _P, _P]),
    "sr_mlp_grad_work": (C.c_int64, []),
    "sr_mlp_backward": (C.c_int, [_P, _P, _P, _P, _I64, _P, _P]),
    "sr_mlp_train": (C.c_int, [_P, _P, _P, _P, _I64, _P, _U64, _I64, _I64, C.c_float, C.c_float,
                               _I32, _D, _D, _P, _P]),
    "sr_mlp_train_work": (C.c_int64, [_I64]),
    "sr_mlp_judge": (C.c_int, [_P, _P, _I32, _I32, _I32, _D, _D, _I32, _D, _P, _P, _P, _P]),
    "sr_mlp_judge_work": (C.c_int64, [_I32, _I32, _I32]),
    "sr_mlp_adam": (C.c_int, [_P, _P, _P, _P, _P, _I64, C.c_float, C.c_float, C.c_float,
                              C.c_float, _P]),
    "sr_mlp_cast": (C.c_int, [_P, _P, _P]),
    "sr_mlp_make_batch": (C.c_int, [_P, _U64, _U64, _I32, _D, _D, _P, _P, _I64, _P]),
    "sr_eval_direct": (C.c_int, [_P, _P, _P, _I32, _P, _I64, _P]),
}

_lib = None


def load(path: str = LIB_PATH):
    """Load libsr.so and attach the signatures.  Raises if it is not built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"libsr.so not found at {path}: build it with "
                           "python -m paper_1409_5574_amd.build")
    lib = C.CDLL(path)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


class SRError(RuntimeError):
    pass


def check(rc: int, what: str):
    if rc != SR_OK:
        msg = load().sr_strerror(rc).decode()
        raise SRError(f"{what} failed: {msg} ({rc})")
