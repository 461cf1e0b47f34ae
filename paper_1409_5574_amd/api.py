"""Thin Python layer over libsr.so: builds the C structs from torch tensors and
calls the entry points with the current HIP stream.  PyTorch provides device
memory and streams only; all arithmetic of the emission path runs in libsr.so.
"""
from __future__ import annotations

import ctypes as C
import dataclasses

import numpy as np
import torch

from . import _lib as L

DEV = "cuda"


def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


def _stream():
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def lib():
    return L.load()


# ------------------------------------------------------------------ tables
class Table:
    """Device spectrum tables (built in FP64 on the GPU)."""

    def __init__(self):
        h = C.c_void_p()
        L.check(lib().sr_table_build(C.byref(h), _stream()), "sr_table_build")
        self.handle = h

    def info(self) -> L.TableInfo:
        inf = L.TableInfo()
        L.check(lib().sr_table_query(self.handle, C.byref(inf)), "sr_table_query")
        return inf

    def free(self):
        if self.handle:
            lib().sr_table_free(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


def eval_F(table: Table, x: torch.Tensor) -> torch.Tensor:
    x = x.contiguous().to(DEV, torch.float32)
    out = torch.empty_like(x)
    L.check(lib().sr_eval_synchrotron_F(table.handle, _ptr(x), _ptr(out), x.numel(), _stream()),
            "sr_eval_synchrotron_F")
    return out


def eval_trial(table: Table, a: torch.Tensor, rate: torch.Tensor, chi: torch.Tensor, kin_cut: bool):
    a = a.contiguous().to(DEV, torch.int32)
    rate = rate.contiguous().to(DEV, torch.float32)
    chi = chi.contiguous().to(DEV, torch.float32)
    dn = torch.empty_like(rate)
    xo = torch.empty_like(rate)
    L.check(lib().sr_eval_trial(table.handle, _ptr(a), _ptr(rate), _ptr(chi), int(kin_cut),
                                _ptr(dn), _ptr(xo), a.numel(), _stream()), "sr_eval_trial")
    return dn, xo


def eval_trial_quantum(table: Table, a: torch.Tensor, rate: torch.Tensor, chi: torch.Tensor):
    """dN = rate Q(x, chi)/S(x) and x of quantum trials (the emission kernel's code)."""
    a = a.contiguous().to(DEV, torch.int32)
    rate = rate.contiguous().to(DEV, torch.float32)
    chi = chi.contiguous().to(DEV, torch.float32)
    dn = torch.empty_like(rate)
    xo = torch.empty_like(rate)
    L.check(lib().sr_eval_trial_quantum(table.handle, _ptr(a), _ptr(rate), _ptr(chi), _ptr(dn),
                                        _ptr(xo), a.numel(), _stream()), "sr_eval_trial_quantum")
    return dn, xo


def philox(ctr: torch.Tensor, seed: int) -> torch.Tensor:
    """ctr: [n,4] int32 (uint32 bit patterns) -> [n,4] int32."""
    ctr = ctr.contiguous().to(DEV, torch.int32)
    out = torch.empty_like(ctr)
    L.check(lib().sr_philox(_ptr(ctr), seed & 0xFFFFFFFFFFFFFFFF, _ptr(out), ctr.shape[0],
                            _stream()), "sr_philox")
    return out


# ------------------------------------------------------------------ state objects
@dataclasses.dataclass
class Particles:
    """SoA particle state on the device (FP32 or FP64)."""
    x: list
    p: list
    w: torch.Tensor
    id: torch.Tensor

    @property
    def n(self):
        return int(self.w.numel())

    @property
    def dtype(self):
        return self.w.dtype

    @staticmethod
    def from_numpy(d: dict, dtype=torch.float32, dim: int = 3) -> "Particles":
        def t(a):
            return torch.from_numpy(np.ascontiguousarray(a)).to(DEV, dtype)
        xs = [t(d["x"]), t(d["y"]), t(d["z"]) if dim == 3 or dim == 0 else None]
        if dim == 2:
            xs[2] = None
        ids = torch.from_numpy(d["id"].astype(np.int64).astype(np.uint32).view(np.int32)).to(DEV)
        return Particles(xs, [t(d["px"]), t(d["py"]), t(d["pz"])], t(d["w"]), ids)

    def to_numpy(self) -> dict:
        out = {k: v.double().cpu().numpy() if v is not None else None
               for k, v in (("x", self.x[0]), ("y", self.x[1]), ("z", self.x[2]))}
        out.update({"px": self.p[0].double().cpu().numpy(), "py": self.p[1].double().cpu().numpy(),
                    "pz": self.p[2].double().cpu().numpy(), "w": self.w.double().cpu().numpy(),
                    "id": self.id.cpu().numpy().view(np.uint32)})
        return out

    def empty_like(self) -> "Particles":
        return Particles([None if a is None else torch.empty_like(a) for a in self.x],
                         [torch.empty_like(a) for a in self.p], torch.empty_like(self.w),
                         torch.empty_like(self.id))

    def struct(self):
        S = L.Particles64 if self.dtype == torch.float64 else L.Particles32
        s = S()
        s.n = self.n
        for a in range(3):
            s.x[a] = None if self.x[a] is None else self.x[a].data_ptr()
            s.p[a] = self.p[a].data_ptr()
        s.w = self.w.data_ptr()
        s.id = self.id.data_ptr()
        return s


def grid_struct(dim: int, n=(1, 1, 1), dx=(1.0, 1.0, 1.0), e0=(0, 0, 0), b0=(0, 0, 0)) -> L.Grid:
    g = L.Grid()
    g.dim = dim
    for a in range(3):
        g.n[a] = int(n[a])
        g.dx[a] = float(dx[a])
        g.e0[a] = float(e0[a])
        g.b0[a] = float(b0[a])
    if dim == 2:
        g.n[2] = 1
    return g


class Fields:
    """Six Yee component arrays (FP32) on the device."""

    def __init__(self, E=None, B=None, ncells: int | None = None):
        if E is None:
            self.e = [torch.empty(ncells, device=DEV, dtype=torch.float32) for _ in range(3)]
            self.b = [torch.empty(ncells, device=DEV, dtype=torch.float32) for _ in range(3)]
        else:
            self.e = [torch.from_numpy(np.ascontiguousarray(a)).to(DEV) for a in E]
            self.b = [torch.from_numpy(np.ascontiguousarray(a)).to(DEV) for a in B]

    def struct(self) -> L.Fields32:
        f = L.Fields32()
        for a in range(3):
            f.e[a] = self.e[a].data_ptr()
            f.b[a] = self.b[a].data_ptr()
        return f


def standing_wave(fields: Fields, grid: L.Grid, a0: float, t: float):
    e = L.P3(*[f.data_ptr() for f in fields.e])
    b = L.P3(*[f.data_ptr() for f in fields.b])
    L.check(lib().sr_field_standing_wave(e, b, C.byref(grid), a0, t, _stream()),
            "sr_field_standing_wave")


def field_step(fields: Fields, grid: L.Grid, dt: float, J: list | None = None):
    """One Yee step of the fields (E and B at whole steps), with current J."""
    e = L.P3(*[f.data_ptr() for f in fields.e])
    b = L.P3(*[f.data_ptr() for f in fields.b])
    j = L.P3(None, None, None) if J is None else L.P3(*[t.data_ptr() for t in J])
    L.check(lib().sr_field_step(e, b, j, C.byref(grid), float(dt), _stream()), "sr_field_step")


def deposit_rho(parts: "Particles", grid: L.Grid, charge: float, rho: torch.Tensor):
    ps = parts.struct()
    L.check(lib().sr_deposit_rho(C.byref(ps), C.byref(grid), float(charge), _ptr(rho), _stream()),
            "sr_deposit_rho")


def deposit_current(parts: "Particles", x_old: list, grid: L.Grid, dt: float, charge: float,
                    J: list, status: torch.Tensor):
    """J += the charge-conserving current of the moves x_old -> parts.x."""
    ps = parts.struct()
    xo = L.P3(*[None if t is None else t.data_ptr() for t in x_old])
    j = L.P3(*[t.data_ptr() for t in J])
    L.check(lib().sr_deposit_current(C.byref(ps), xo, C.byref(grid), float(dt), float(charge), j,
                                     _ptr(status), _stream()), "sr_deposit_current")


def photon_advance(photons: "PhotonBuffer", n: int, grid: L.Grid, dt: float,
                   start: torch.Tensor | None = None):
    cs = L.Chunking()
    cs.n_chunks = n_chunks_uniform(n) if start is None else start.numel() - 1
    cs.start = None if start is None else start.data_ptr()
    phs = photons.struct()
    L.check(lib().sr_photon_advance(C.byref(phs), C.byref(cs), n, C.byref(grid), float(dt),
                                    _stream()), "sr_photon_advance")


def n_chunks_uniform(n: int) -> int:
    return (n + L.SR_CHUNK - 1) // L.SR_CHUNK


class PhotonBuffer:
    def __init__(self, n: int, per_particle: int, n_chunks: int | None = None, dim: int = 3,
                 with_k: bool = True, with_step: bool = False):
        n_chunks = n_chunks_uniform(n) if n_chunks is None else n_chunks
        cap = max(n * per_particle, 1)
        f = dict(device=DEV, dtype=torch.float32)
        self.per_particle = per_particle
        self.n_chunks = n_chunks
        self.seg_count = torch.zeros(max(n_chunks, 1), device=DEV, dtype=torch.int32)
        self.eps = torch.empty(cap, **f)
        self.w = torch.empty(cap, **f)
        self.dir = [torch.empty(cap, **f) for _ in range(3)]
        self.pos = [torch.empty(cap, **f) for _ in range(3 if dim != 2 else 2)] + \
            ([None] if dim == 2 else [])
        self.parent = torch.empty(cap, device=DEV, dtype=torch.int32)
        self.k = torch.empty(cap, device=DEV, dtype=torch.uint8) if with_k else None
        self.step = torch.empty(cap, device=DEV, dtype=torch.int32) if with_step else None

    def struct(self) -> L.PhotonBuf:
        s = L.PhotonBuf()
        s.per_particle = self.per_particle
        s.seg_count = self.seg_count.data_ptr()
        s.eps = self.eps.data_ptr()
        s.w = self.w.data_ptr()
        for a in range(3):
            s.dir[a] = self.dir[a].data_ptr()
            s.pos[a] = None if self.pos[a] is None else self.pos[a].data_ptr()
        s.parent = self.parent.data_ptr()
        s.k = None if self.k is None else self.k.data_ptr()
        s.step = None if self.step is None else self.step.data_ptr()
        return s

    def gather(self, n: int, start: torch.Tensor | None = None) -> dict:
        """Copy the stored photons of every segment to host numpy arrays."""
        cnt = self.seg_count.cpu().numpy().view(np.uint32).astype(np.int64)
        if start is None:
            s = np.arange(self.n_chunks, dtype=np.int64) * L.SR_CHUNK
            e = np.minimum(s + L.SR_CHUNK, n)
        else:
            st = start.cpu().numpy()
            s, e = st[:-1], st[1:]
        cap = (e - s) * self.per_particle
        stored = np.minimum(cnt, cap)
        idx = np.concatenate([np.arange(b * self.per_particle, b * self.per_particle + c)
                              for b, c in zip(s, stored)]) if stored.sum() else np.zeros(0, np.int64)
        it = torch.from_numpy(idx).to(DEV)

        def g(t):
            return None if t is None else t[it].cpu().numpy()
        out = {"eps": g(self.eps), "w": g(self.w),
               "dir": np.stack([g(d) for d in self.dir], 1) if len(idx) else np.zeros((0, 3)),
               "pos": np.stack([g(d) if d is not None else np.zeros(len(idx), np.float32)
                                for d in self.pos], 1) if len(idx) else np.zeros((0, 3)),
               "parent": g(self.parent).view(np.uint32) if len(idx) else np.zeros(0, np.uint32),
               "k": g(self.k) if self.k is not None else None,
               "count": int(cnt.sum()), "stored": int(stored.sum())}
        return out


class LedgerBuf:
    def __init__(self, n_rows: int, n_chunks: int, steps_per_call: int = 1):
        """Ledger rows and partials; steps_per_call > 1 sizes the partials for
        sr_gather_push_emit_steps with that many steps."""
        self.rows = torch.zeros((max(n_rows, 1), L.SR_LEDGER_COLS), device=DEV, dtype=torch.float64)
        plen = int(lib().sr_ledger_partials(n_chunks))
        if steps_per_call > 1:
            plen = max(plen, int(lib().sr_ledger_partials_steps(n_chunks, steps_per_call)))
        self.partials = torch.zeros(max(plen, 1), device=DEV, dtype=torch.float64)
        self.status = torch.zeros(1, device=DEV, dtype=torch.int32)
        self.n_rows = n_rows

    def struct(self) -> L.Ledger:
        s = L.Ledger()
        s.rows = self.rows.data_ptr()
        s.n_rows = self.n_rows
        s.partials = self.partials.data_ptr()
        s.partials_len = self.partials.numel()
        s.status = self.status.data_ptr()
        return s

    def row(self, r: int) -> np.ndarray:
        out = np.zeros(L.SR_LEDGER_COLS)
        s = self.struct()
        L.check(lib().sr_energy_ledger(C.byref(s), r, out.ctypes.data_as(C.c_void_p), _stream()),
                "sr_energy_ledger")
        return out

    def read_status(self, clear: bool = False) -> int:
        v = C.c_uint32()
        s = self.struct()
        L.check(lib().sr_status(C.byref(s), C.byref(v), int(clear), _stream()), "sr_status")
        return v.value


def params_struct(hbar_n, alpha, n_samples=1, sampler=L.SR_SAMPLER_S, recoil=L.SR_RECOIL_PHOTON,
                  dn_policy=L.SR_DN_WEIGHT, kin_cut=False, push_position=True,
                  mlp: "Mlp | None" = None, omega_grid: float = 0.0,
                  gather: int = L.SR_GATHER_DIRECT) -> L.Params:
    """Step parameters.  With the learned sampler the network must have been
    trained with the same kinematic-cut setting (its draws are x of the cut or
    uncut spectrum), and when its fallback map sends every chi bin to the table
    the table sampler is dispatched instead: the same decisions and draws,
    without the network's LDS and compaction."""
    if sampler == L.SR_SAMPLER_MLP:
        if mlp is None:
            raise ValueError("the learned sampler needs its network (mlp=)")
        if mlp.kin_cut is None:
            raise ValueError("the network has not been trained")
        if bool(mlp.kin_cut) != bool(kin_cut):
            raise ValueError(f"the network was trained with kin_cut={mlp.kin_cut}, "
                             f"the step asks for kin_cut={bool(kin_cut)}")
        if mlp.all_on_table():
            sampler, mlp = L.SR_SAMPLER_TABLE, None
    return L.Params(float(hbar_n), float(alpha), int(n_samples), int(sampler), int(recoil),
                    int(dn_policy), int(bool(kin_cut)), int(bool(push_position)),
                    None if mlp is None else mlp.params.data_ptr(),
                    None if mlp is None else mlp.fallback.data_ptr(), float(omega_grid),
                    int(gather), 0)


def eval_direct(table: Table, a: torch.Tensor, chi: torch.Tensor, kin_cut: bool) -> torch.Tensor:
    a = a.contiguous().to(DEV, torch.int32)
    chi = chi.contiguous().to(DEV, torch.float32)
    out = torch.empty_like(chi)
    L.check(lib().sr_eval_direct(table.handle, _ptr(a), _ptr(chi), int(kin_cut), _ptr(out),
                                 a.numel(), _stream()), "sr_eval_direct")
    return out


def mlp_init(seed: int) -> np.ndarray:
    """Initial FP32 parameters in the flat sr_mlp layout (W1[64][2], b1, W2[64][64],
    b2, W3[64][64], b3, W4[64], b4): normal weights with variance 2/fan_in
    (1/fan_in for the linear output layer), zero biases."""
    rng = np.random.default_rng(seed)
    h = 64
    parts = [rng.normal(0.0, 1.0, h * 2), np.zeros(h),
             rng.normal(0.0, np.sqrt(2.0 / h), h * h), np.zeros(h),
             rng.normal(0.0, np.sqrt(2.0 / h), h * h), np.zeros(h),
             rng.normal(0.0, np.sqrt(1.0 / h), h), np.zeros(1)]
    flat = np.concatenate(parts).astype(np.float32)
    assert flat.size == L.SR_MLP_PARAMS
    return flat


class Mlp:
    """The MLP surrogate: FP32 master weights, Adam moments and the bfloat16
    copy the kernels read, all on the device."""

    def __init__(self, master: np.ndarray):
        assert master.size == L.SR_MLP_PARAMS
        self.master = torch.from_numpy(np.asarray(master, np.float32)).to(DEV)
        self.params = torch.empty(L.SR_MLP_PARAMS, device=DEV, dtype=torch.bfloat16)
        self.m = torch.zeros_like(self.master)
        self.v = torch.zeros_like(self.master)
        self.grads = torch.zeros_like(self.master)
        self.work = torch.empty(int(lib().sr_mlp_grad_work()), device=DEV, dtype=torch.float32)
        # every chi bin on the table until the judge admits the network
        self.fallback = torch.ones(L.SR_MLP_FALLBACK_BINS, device=DEV, dtype=torch.uint8)
        self.fallback_host = np.ones(L.SR_MLP_FALLBACK_BINS, np.uint8)
        self.kin_cut = None          # the cut setting the network was trained with
        self.t = 0
        L.check(lib().sr_mlp_cast(_ptr(self.master), _ptr(self.params), _stream()), "sr_mlp_cast")

    def forward(self, feats: torch.Tensor) -> torch.Tensor:
        feats = feats.contiguous().to(DEV, torch.float32)
        out = torch.empty(feats.shape[0], device=DEV, dtype=torch.float32)
        L.check(lib().sr_mlp_forward(_ptr(self.params), _ptr(feats), _ptr(out), feats.shape[0],
                                     _stream()), "sr_mlp_forward")
        return out

    def mse_grad(self, feats: torch.Tensor, target: torch.Tensor) -> torch.Tensor:
        L.check(lib().sr_mlp_mse_grad(_ptr(self.params), _ptr(feats), _ptr(target),
                                      feats.shape[0], _ptr(self.grads), _ptr(self.work),
                                      _stream()), "sr_mlp_mse_grad")
        return self.grads

    def adam(self, lr: float, beta1=0.9, beta2=0.999, eps=1e-8):
        self.t += 1
        L.check(lib().sr_mlp_adam(_ptr(self.master), _ptr(self.params), _ptr(self.grads),
                                  _ptr(self.m), _ptr(self.v), self.t, lr, beta1, beta2, eps,
                                  _stream()), "sr_mlp_adam")

    def set_fallback(self, fb):
        """Set the per-chi-bin fallback map (1: that bin draws from the table)."""
        fb = torch.as_tensor(fb).to(torch.uint8).reshape(-1)
        assert fb.numel() == L.SR_MLP_FALLBACK_BINS
        self.fallback.copy_(fb.to(DEV))
        self.fallback_host = fb.cpu().numpy().astype(np.uint8)

    def all_on_table(self) -> bool:
        return bool(np.all(self.fallback_host != 0))

    def backward(self, feats: torch.Tensor, dout: torch.Tensor) -> torch.Tensor:
        """Gradient of sum dout * network(feats) with respect to the parameters."""
        feats = feats.contiguous().to(DEV, torch.float32)
        dout = dout.contiguous().to(DEV, torch.float32)
        grads = torch.empty_like(self.master)
        L.check(lib().sr_mlp_backward(_ptr(self.params), _ptr(feats), _ptr(dout), _ptr(grads),
                                      feats.shape[0], _ptr(self.work), _stream()), "sr_mlp_backward")
        return grads

    def train(self, table: Table, steps: int, batch: int, lr: float, seed: int = 0x5A11,
              kin_cut: bool = True, lo: float = -4.0, hi: float = 2.0, lr_final: float | None = None):
        """Adam on fresh batches of table-generated pairs with a cosine-decayed
        learning rate, the whole loop enqueued by the library (sr_mlp_train)."""
        if self.kin_cut is not None and bool(self.kin_cut) != bool(kin_cut):
            raise ValueError("the network was trained with the other kinematic-cut setting")
        self.kin_cut = bool(kin_cut)
        lr_final = lr * 0.01 if lr_final is None else lr_final
        work = torch.empty(int(lib().sr_mlp_train_work(batch)), device=DEV, dtype=torch.float32)
        L.check(lib().sr_mlp_train(_ptr(self.master), _ptr(self.params), _ptr(self.m), _ptr(self.v),
                                   self.t, table.handle, seed, steps, batch, lr, lr_final,
                                   int(kin_cut), lo, hi, _ptr(work), _stream()), "sr_mlp_train")
        self.t += steps

    def judge(self, table: Table, kin_cut: bool = True, n_u: int = 1 << 14, chi_per_bin: int = 8,
              x_lo: float = 1e-4, x_hi: float = 16.4, n_xbins: int = 64, tol: float = 1e-3):
        """The library's judge (sr_mlp_judge): the binned-spectrum error of the
        network against the table sampler per bin of log10 chi, on a stratified
        grid of u and chi; bins above `tol` are switched to the table.  Returns
        the errors (host numpy)."""
        nb = L.SR_MLP_FALLBACK_BINS
        work = torch.empty(int(lib().sr_mlp_judge_work(n_u, chi_per_bin, n_xbins)), device=DEV,
                           dtype=torch.float32)
        err = torch.empty(nb, device=DEV, dtype=torch.float64)
        fb = torch.empty(nb, device=DEV, dtype=torch.uint8)
        L.check(lib().sr_mlp_judge(_ptr(self.params), table.handle, int(kin_cut), n_u, chi_per_bin,
                                   x_lo, x_hi, n_xbins, tol, _ptr(err), _ptr(fb), _ptr(work),
                                   _stream()), "sr_mlp_judge")
        self.set_fallback(fb)
        return err.cpu().numpy()

    def make_batch(self, table: Table, seed: int, batch_index: int, M: int, kin_cut=True,
                   lo=-4.0, hi=2.0):
        feats = torch.empty((M, 2), device=DEV, dtype=torch.float32)
        target = torch.empty(M, device=DEV, dtype=torch.float32)
        L.check(lib().sr_mlp_make_batch(table.handle, seed, batch_index, int(kin_cut), lo, hi,
                                        _ptr(feats), _ptr(target), M, _stream()),
                "sr_mlp_make_batch")
        return feats, target


def gather_push_emit(parts: Particles, fields: Fields | None, grid: L.Grid, dt: float, seed: int,
                     step: int, prm: L.Params, table: Table, photons: PhotonBuffer,
                     ledger: LedgerBuf, row: int | None, start: torch.Tensor | None = None,
                     structs: tuple | None = None, events: tuple | None = None):
    """One emission step; with row set, also reduce the ledger into that row.
    `structs` may hold pre-built (parts, fields, chunking, photons, ledger) C
    structs to avoid rebuilding them every call.  `events`: a (start, stop)
    pair of recorded torch.cuda.Event(enable_timing=True) that the kernel's own
    dispatch re-records at its start and end (FP32 path)."""
    if structs is None:
        structs = make_structs(parts, fields, photons, ledger, start)
    ps, fs, cs, phs, ls = structs
    args = (C.byref(ps), C.byref(fs) if fs is not None else None, C.byref(grid), float(dt),
            seed & 0xFFFFFFFFFFFFFFFF, int(step), C.byref(prm), table.handle, C.byref(cs),
            C.byref(phs), C.byref(ls))
    if events is not None:
        if parts.dtype != torch.float32:
            raise ValueError("timed launches exist for the FP32 path only")
        rc = lib().sr_gather_push_emit_timed(*args, C.c_void_p(events[0].cuda_event),
                                             C.c_void_p(events[1].cuda_event), _stream())
    else:
        fn = (lib().sr_gather_push_emit_f64 if parts.dtype == torch.float64
              else lib().sr_gather_push_emit)
        rc = fn(*args, _stream())
    L.check(rc, "sr_gather_push_emit")
    if row is not None:
        ledger_reduce(ledger, cs.n_chunks, row, ls)


def gather_push_emit_steps(parts: Particles, grid: L.Grid, dt: float, seed: int, step0: int,
                           n_steps: int, prm: L.Params, table: Table, photons: PhotonBuffer,
                           ledger: "LedgerBuf", structs: tuple | None = None):
    """n_steps emission steps in one launch (uniform fields): ledger rows
    0 .. n_steps-1 receive the steps step0 ...; the photon segments hold the
    photons of every step (with their step index if the buffer has one)."""
    if structs is None:
        structs = make_structs(parts, None, photons, ledger)
    ps, _, _, phs, ls = structs
    L.check(lib().sr_gather_push_emit_steps(C.byref(ps), C.byref(grid), float(dt),
                                            seed & 0xFFFFFFFFFFFFFFFF, int(step0), int(n_steps),
                                            C.byref(prm), table.handle, C.byref(phs), C.byref(ls),
                                            _stream()), "sr_gather_push_emit_steps")


def gather_push_emit_noalloc(parts: Particles, fields: Fields | None, grid: L.Grid, dt: float,
                             seed: int, step: int, prm: L.Params, table: Table,
                             photons: PhotonBuffer, ledger_row: torch.Tensor,
                             status: torch.Tensor, start: torch.Tensor | None = None):
    """sr_gather_push_emit_noalloc: one emission step and its ledger row
    (device float64[SR_LEDGER_COLS]); the step's partial rows live in the
    library's own device array, so the call allocates nothing."""
    if parts.dtype != torch.float32:
        raise ValueError("the no-allocation step exists for the FP32 path only")
    if ledger_row.dtype != torch.float64 or ledger_row.numel() < L.SR_LEDGER_COLS:
        raise ValueError("ledger_row: a device float64 tensor of SR_LEDGER_COLS values")
    if status.numel() < 1 or status.element_size() != 4:
        raise ValueError("status: a device 32-bit word")
    cs = L.Chunking()
    cs.n_chunks = n_chunks_uniform(parts.n) if start is None else start.numel() - 1
    cs.start = None if start is None else start.data_ptr()
    ps = parts.struct()
    fs = fields.struct() if fields is not None else None
    phs = photons.struct()
    L.check(lib().sr_gather_push_emit_noalloc(
        C.byref(ps), C.byref(fs) if fs is not None else None, C.byref(grid), float(dt),
        seed & 0xFFFFFFFFFFFFFFFF, int(step), C.byref(prm), table.handle, C.byref(cs),
        C.byref(phs), _ptr(ledger_row), _ptr(status), _stream()), "sr_gather_push_emit_noalloc")


def eval_push(parts: Particles, fields: Fields | None, grid: L.Grid, dt: float, hbar_n: float,
              alpha: float) -> dict:
    """H_eff, chi and the mean gamma of one push of every particle (the step's
    own gather / Boris / H_eff code), FP64 device arrays; particles untouched."""
    n = parts.n
    out = {k: torch.empty(max(n, 1), device=DEV, dtype=torch.float64)
           for k in ("heff", "chi", "gamma_bar")}
    prm = params_struct(hbar_n, alpha)
    ps = parts.struct()
    fs = fields.struct() if fields is not None else None
    fn = lib().sr_eval_push_f64 if parts.dtype == torch.float64 else lib().sr_eval_push
    L.check(fn(C.byref(ps), C.byref(fs) if fs is not None else None, C.byref(grid), float(dt),
               C.byref(prm), _ptr(out["heff"]), _ptr(out["chi"]), _ptr(out["gamma_bar"]),
               _stream()), "sr_eval_push")
    return {k: v[:n] for k, v in out.items()}


def validity(parts: Particles, fields: Fields | None, grid: L.Grid, dt: float, hbar_n: float,
             alpha: float, tau_em: float, want_flags: bool = True):
    """Validity flags (uint8 per particle, SR_VALID_* bits, or None) and the six
    weighted sums of sr_validity (host numpy)."""
    n = parts.n
    flags = torch.empty(max(n, 1), device=DEV, dtype=torch.uint8) if want_flags else None
    sums = torch.empty(L.SR_VALID_SUMS, device=DEV, dtype=torch.float64)
    nw = int(lib().sr_validity_work(n))
    work = torch.empty(max(nw, 1), device=DEV, dtype=torch.float64)
    prm = params_struct(hbar_n, alpha)
    ps = parts.struct()
    fs = fields.struct() if fields is not None else None
    L.check(lib().sr_validity(C.byref(ps), C.byref(fs) if fs is not None else None, C.byref(grid),
                              float(dt), C.byref(prm), float(tau_em), _ptr(flags), _ptr(sums),
                              _ptr(work), _stream()), "sr_validity")
    return (None if flags is None else flags[:n]), sums.cpu().numpy()


def ledger_reduce(ledger: "LedgerBuf", n_chunks: int, row: int, ls=None):
    ls = ledger.struct() if ls is None else ls
    L.check(lib().sr_ledger_reduce(C.byref(ls), int(n_chunks), int(row), _stream()),
            "sr_ledger_reduce")


def make_structs(parts, fields, photons, ledger, start=None):
    cs = L.Chunking()
    if start is None:
        cs.n_chunks = n_chunks_uniform(parts.n)
        cs.start = None
    else:
        cs.n_chunks = start.numel() - 1
        cs.start = start.data_ptr()
    return (parts.struct(), fields.struct() if fields is not None else None, cs, photons.struct(),
            ledger.struct())


def spectrum_histogram(photons: PhotonBuffer, n: int, eps_lo: float, eps_hi: float, n_bins: int,
                       hist: torch.Tensor, work: torch.Tensor, start: torch.Tensor | None = None):
    cs = L.Chunking()
    cs.n_chunks = n_chunks_uniform(n) if start is None else start.numel() - 1
    cs.start = None if start is None else start.data_ptr()
    phs = photons.struct()
    L.check(lib().sr_spectrum_histogram(C.byref(phs), C.byref(cs), n, eps_lo, eps_hi, n_bins,
                                        _ptr(hist), _ptr(work), _stream()), "sr_spectrum_histogram")


def step_epilogue(ledger: "LedgerBuf", n_chunks: int, row: int, photons: PhotonBuffer, n: int,
                  eps_lo: float, eps_hi: float, n_bins: int, hist: torch.Tensor,
                  work: torch.Tensor, start: torch.Tensor | None = None, ls=None):
    """ledger_reduce(ledger, n_chunks, row) and spectrum_histogram(photons, n,
    ...) in two launches instead of four (same results)."""
    ls = ledger.struct() if ls is None else ls
    cs = L.Chunking()
    cs.n_chunks = n_chunks_uniform(n) if start is None else start.numel() - 1
    cs.start = None if start is None else start.data_ptr()
    phs = photons.struct()
    L.check(lib().sr_step_epilogue(C.byref(ls), int(n_chunks), int(row), C.byref(phs), C.byref(cs),
                                   n, eps_lo, eps_hi, n_bins, _ptr(hist), _ptr(work), _stream()),
            "sr_step_epilogue")


def angular_histogram(photons: PhotonBuffer, n: int, axis, ref, n_theta: int, n_phi: int,
                      hist: torch.Tensor, work: torch.Tensor, start: torch.Tensor | None = None):
    """hist[n_theta*n_phi + 1] += energy-weighted (theta, phi) map of the stored
    photons over the front hemisphere around `axis` (last entry: back hemisphere)."""
    cs = L.Chunking()
    cs.n_chunks = n_chunks_uniform(n) if start is None else start.numel() - 1
    cs.start = None if start is None else start.data_ptr()
    phs = photons.struct()
    ax = (C.c_double * 3)(*[float(v) for v in axis])
    rf = (C.c_double * 3)(*[float(v) for v in ref])
    L.check(lib().sr_angular_histogram(C.byref(phs), C.byref(cs), n, ax, rf, int(n_theta),
                                       int(n_phi), _ptr(hist), _ptr(work), _stream()),
            "sr_angular_histogram")


def angular_work(n_theta: int, n_phi: int) -> torch.Tensor:
    nw = int(lib().sr_angular_work(n_theta, n_phi))
    if nw < 0:
        raise L.SRError("sr_angular_work: bad bin counts")
    return torch.zeros(nw, device=DEV, dtype=torch.float64)


def hist_work(n_bins: int) -> torch.Tensor:
    return torch.zeros(int(lib().sr_hist_work(n_bins)), device=DEV, dtype=torch.float64)


def sort_work(grid: L.Grid, tile, n: int) -> torch.Tensor:
    t = (C.c_int32 * 3)(*tile)
    nbytes = int(lib().sr_sort_work(C.byref(grid), t, n))
    if nbytes < 0:
        raise L.SRError("sr_sort_work: bad grid or tile")
    return torch.empty(max(nbytes, 4), device=DEV, dtype=torch.uint8)


def sort_particles(src: Particles, dst: Particles, grid: L.Grid, tile, work: torch.Tensor):
    t = (C.c_int32 * 3)(*tile)
    s, d = src.struct(), dst.struct()
    L.check(lib().sr_sort_particles(C.byref(s), C.byref(d), C.byref(grid), t, _ptr(work),
                                    _stream()), "sr_sort_particles")
