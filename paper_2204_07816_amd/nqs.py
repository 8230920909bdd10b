"""Thin Python binding of libnqs (the C ABI in include/nqs.h).

Argument marshalling only: torch tensors supply device memory and the HIP
stream; every step of the computation runs in the library's HIP kernels.
There is no CPU fallback: when ``libnqs.so`` is missing or cannot be loaded,
every entry point raises.
"""
from __future__ import annotations

import ctypes
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libnqs.so")

FP64, FP32, BF16, BF16X3 = 0, 1, 2, 3
AUTO, FULL, INCREMENTAL = 0, 1, 2
_DTYPES = {"fp64": FP64, "fp32": FP32, "bf16": BF16, "bf16x3": BF16X3}
_MODES = {"auto": AUTO, "full": FULL, "incremental": INCREMENTAL}

STATUS = {
    0: "NQS_OK", 1: "NQS_E_ARG", 2: "NQS_E_LATTICE", 3: "NQS_E_SPEC", 4: "NQS_E_NPARAMS",
    5: "NQS_E_SPIN", 6: "NQS_E_NONFINITE", 7: "NQS_E_NOMEM", 8: "NQS_E_WORKSPACE",
    9: "NQS_E_HIP", 10: "NQS_E_UNSUPPORTED",
}


class NqsError(RuntimeError):
    def __init__(self, code: int, where: str):
        self.code = code
        super().__init__(f"{where}: {STATUS.get(code, code)} ({_status_str(code)})")


class CnnSpec(ctypes.Structure):
    _fields_ = [("n_layers", ctypes.c_int32), ("channels", ctypes.c_int32),
                ("marshall_sign", ctypes.c_int32), ("conv_dtype", ctypes.c_int32)]


class ElocJob(ctypes.Structure):
    _fields_ = [("ctx", ctypes.c_void_p), ("spins", ctypes.c_void_p), ("B", ctypes.c_int64),
                ("e_loc", ctypes.c_void_p)]


_lib = None


def load():
    """Load libnqs.so (torch is imported first so both share one HIP runtime)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"libnqs.so not found at {LIB_PATH}: run __graft_entry__.build() "
                           "(hipcc for gfx950); there is no fallback")
    lib = ctypes.CDLL(LIB_PATH)
    vp, i32, i64, d = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
    P = ctypes.POINTER
    sig = {
        "nqs_create": [i32, d, d, P(CnnSpec), vp, i64, P(vp)],
        "nqs_create_tj": [i32, d, d, P(CnnSpec), vp, i64, P(vp)],
        "nqs_create_cnn1": [i32, d, d, i32, i32, i32, vp, i64, P(vp)],
        "nqs_create_cnn1_tj": [i32, d, d, i32, i32, i32, vp, i64, P(vp)],
        "nqs_create_cnn2_tj": [i32, d, d, i32, i32, i32, vp, i64, P(vp)],
        "nqs_mfma_rate": [i32, i64, i32, P(d), P(d), vp],
        "nqs_destroy": [vp],
        "nqs_num_params": [vp, P(i64)],
        "nqs_set_weights": [vp, vp, i64],
        "nqs_reserve": [vp, i64, i32],
        "nqs_log_psi": [vp, vp, i64, vp, vp, vp],
        "nqs_local_energy": [vp, vp, i64, vp, i32, vp],
        "nqs_energy_stats": [vp, vp, i64, vp, vp],
        "nqs_log_deriv": [vp, vp, i64, vp, i32, vp],
        "nqs_sr_solve": [vp, vp, i32, vp, i64, d, i32, vp, vp, vp],
        "nqs_sr_solve_recompute": [vp, vp, i32, vp, i64, d, i32, i64, vp, vp, vp],
        "nqs_sr_solve_noalloc": [vp, vp, i32, vp, i64, d, i32, vp, vp, vp],
        "nqs_connected": [vp, vp, i64, vp, vp, vp, vp, i64, vp, vp],
        "nqs_log_ratios": [vp, vp, i64, i32, vp, i64, vp],
        "nqs_local_energy_multi": [vp, i32, i32, vp],
        "nqs_mcmc": [vp, vp, i64, i32, vp, vp, vp, i32, vp],
        "nqs_update_weights": [vp, vp, d, vp],
        "nqs_get_weights": [vp, vp, i64],
        "nqs_set_weights_device": [vp, vp, vp],
        "nqs_auto_mode": [vp, P(i32)],
        "nqs_autotune": [vp, vp, i64, P(i32), vp],
        "nqs_tune_key": [i32, i32, i32, i32, d, ctypes.c_char_p, i64],
        "nqs_tune_lookup": [ctypes.c_char_p, ctypes.c_char_p, P(i32), P(i32), P(i32), P(i32),
                            P(i32)],
        "nqs_get_error": [vp, P(i32)],
        "nqs_enable_timing": [vp, i32],
        "nqs_kernel_time": [vp, P(d), P(i64)],
    }
    for name, args in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = ctypes.c_int
    lib.nqs_status_str.argtypes = [ctypes.c_int]
    lib.nqs_status_str.restype = ctypes.c_char_p
    _lib = lib
    return lib


def _status_str(code: int) -> str:
    try:
        return load().nqs_status_str(code).decode()
    except Exception:  # noqa: BLE001 - message only
        return "?"


def _check(code: int, where: str):
    if code != 0:
        raise NqsError(code, where)


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _dev(t: torch.Tensor, dtype: torch.dtype, name: str):
    if not isinstance(t, torch.Tensor) or t.device.type != "cuda":
        raise TypeError(f"{name} must be a CUDA (HIP) tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    return ctypes.c_void_p(t.data_ptr())


def num_params(K: int, C: int) -> int:
    return (C * 9 + C) + (K - 1) * (C * C * 9 + C)


class Context:
    """One lattice + network (nqs_create / nqs_create_tj / nqs_create_cnn1 /
    nqs_create_cnn1_tj / nqs_create_cnn2_tj / nqs_destroy)."""

    def __init__(self, L: int, J1: float, J2: float, K: int, C: int, weights,
                 dtype: str = "fp64", marshall_sign: bool = True, *,
                 tj_hop: float | None = None, net: str = "lncosh"):
        lib = load()
        w = torch.as_tensor(weights, dtype=torch.float64).contiguous().cpu()
        spec = CnnSpec(K, C, 1 if marshall_sign else 0, _DTYPES[dtype])
        h = ctypes.c_void_p()
        if net == "cnn1":
            if dtype != "fp64":
                raise ValueError("CNN1 contexts are FP64")
            if tj_hop is None:
                _check(lib.nqs_create_cnn1(L, J1, J2, K, C, 1 if marshall_sign else 0,
                                           ctypes.c_void_p(w.data_ptr()), w.numel(),
                                           ctypes.byref(h)), "nqs_create_cnn1")
            else:
                if J2 != 0.0:
                    raise ValueError("t-J contexts have no next-nearest coupling")
                _check(lib.nqs_create_cnn1_tj(L, tj_hop, J1, K, C, 1 if marshall_sign else 0,
                                              ctypes.c_void_p(w.data_ptr()), w.numel(),
                                              ctypes.byref(h)), "nqs_create_cnn1_tj")
        elif net == "cnn2":
            if dtype != "fp64" or tj_hop is None or J2 != 0.0:
                raise ValueError("CNN2 contexts are FP64 t-J contexts")
            _check(lib.nqs_create_cnn2_tj(L, tj_hop, J1, K, C, 1 if marshall_sign else 0,
                                          ctypes.c_void_p(w.data_ptr()), w.numel(),
                                          ctypes.byref(h)), "nqs_create_cnn2_tj")
        elif tj_hop is None:
            _check(lib.nqs_create(L, J1, J2, ctypes.byref(spec), ctypes.c_void_p(w.data_ptr()),
                                  w.numel(), ctypes.byref(h)), "nqs_create")
        else:
            _check(lib.nqs_create_tj(L, tj_hop, J1, ctypes.byref(spec),
                                     ctypes.c_void_p(w.data_ptr()), w.numel(), ctypes.byref(h)),
                   "nqs_create_tj")
        self._h = h
        self.L, self.J1, self.J2, self.K, self.C, self.dtype = L, J1, J2, K, C, dtype
        self.model = "spin" if tj_hop is None else "tj"
        self.net = net
        self.t = tj_hop
        self.P = self.num_params()

    @classmethod
    def cnn1(cls, L: int, J1: float, J2: float, blocks: int, C: int, weights,
             marshall_sign: bool = True) -> "Context":
        """A CNN1 context (nqs_create_cnn1), FP64: `blocks` blocks of C channels."""
        return cls(L, J1, J2, blocks, C, weights, "fp64", marshall_sign, net="cnn1")

    @classmethod
    def cnn1_tj(cls, L: int, t: float, J: float, blocks: int, C: int, weights,
                marshall_sign: bool = True) -> "Context":
        """A t-J context with the CNN1 amplitude (nqs_create_cnn1_tj), FP64."""
        return cls(L, J, 0.0, blocks, C, weights, "fp64", marshall_sign, tj_hop=t, net="cnn1")

    @classmethod
    def cnn2_tj(cls, L: int, t: float, J: float, blocks: int, C: int, weights,
                marshall_sign: bool = True) -> "Context":
        """A t-J context with the CNN2 amplitude (nqs_create_cnn2_tj), FP64,
        C = 16 or 32."""
        return cls(L, J, 0.0, blocks, C, weights, "fp64", marshall_sign, tj_hop=t, net="cnn2")

    @classmethod
    def tj(cls, L: int, t: float, J: float, K: int, C: int, weights, dtype: str = "fp64",
           marshall_sign: bool = True) -> "Context":
        """A t-J context (nqs_create_tj): site values +1 up, -1 down, 0 hole."""
        return cls(L, J, 0.0, K, C, weights, dtype, marshall_sign, tj_hop=t)

    @property
    def handle(self):
        return self._h

    def close(self):
        if getattr(self, "_h", None) and self._h.value:
            load().nqs_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:  # noqa: BLE001 - interpreter shutdown
            pass

    def num_params(self) -> int:
        p = ctypes.c_int64()
        _check(load().nqs_num_params(self._h, ctypes.byref(p)), "nqs_num_params")
        return p.value

    def set_weights(self, weights):
        w = torch.as_tensor(weights, dtype=torch.float64).contiguous().cpu()
        _check(load().nqs_set_weights(self._h, ctypes.c_void_p(w.data_ptr()), w.numel()),
               "nqs_set_weights")

    def update_weights(self, dtheta, scale: float):
        """theta <- theta + scale * dtheta on the device (dtheta FP64 [P] tensor)."""
        if dtheta.numel() != self.P:
            raise ValueError("dtheta must hold P values")
        _check(load().nqs_update_weights(self._h, _dev(dtheta, torch.float64, "dtheta"),
                                         float(scale), _stream()), "nqs_update_weights")

    def set_weights_device(self, theta):
        """theta (FP64 [P] device tensor, canonical order) becomes the weights,
        on the current stream, with no host round trip or synchronisation."""
        if theta.numel() != self.P:
            raise ValueError("theta must hold P values")
        _check(load().nqs_set_weights_device(self._h, _dev(theta, torch.float64, "theta"),
                                             _stream()), "nqs_set_weights_device")

    def get_weights(self):
        """The current canonical weights (numpy FP64 [P])."""
        import numpy as np
        out = np.empty(self.P, np.float64)
        _check(load().nqs_get_weights(self._h, out.ctypes.data_as(ctypes.c_void_p), self.P),
               "nqs_get_weights")
        return out

    def reserve(self, B_max: int, mode: str = "auto"):
        _check(load().nqs_reserve(self._h, B_max, _MODES[mode]), "nqs_reserve")

    def auto_mode(self) -> str:
        m = ctypes.c_int32()
        _check(load().nqs_auto_mode(self._h, ctypes.byref(m)), "nqs_auto_mode")
        return {v: k for k, v in _MODES.items()}[m.value]

    def autotune(self, spins) -> str:
        """Time the exchanged-configuration pass in every available form on these
        samples; AUTO uses the fastest from then on (and the tune cache keeps it)."""
        sp, B = self._spins(spins)
        m = ctypes.c_int32()
        _check(load().nqs_autotune(self._h, sp, B, ctypes.byref(m), _stream()), "nqs_autotune")
        return {v: k for k, v in _MODES.items()}[m.value]

    def _spins(self, spins):
        sp = _dev(spins, torch.int8, "spins")
        B = spins.numel() // (self.L * self.L)
        if spins.numel() != B * self.L * self.L:
            raise ValueError("spins must hold B*L*L values")
        return sp, B

    def log_psi(self, spins, with_sign: bool = True):
        sp, B = self._spins(spins)
        la = torch.empty(B, dtype=torch.float64, device=spins.device)
        sg = torch.empty(B, dtype=torch.int8, device=spins.device) if with_sign else None
        _check(load().nqs_log_psi(self._h, sp, B, ctypes.c_void_p(la.data_ptr()),
                                  ctypes.c_void_p(sg.data_ptr() if sg is not None else 0),
                                  _stream()), "nqs_log_psi")
        return (la, sg) if with_sign else la

    def local_energy(self, spins, mode: str = "auto", out=None):
        sp, B = self._spins(spins)
        e = out if out is not None else torch.empty(B, dtype=torch.float64, device=spins.device)
        _check(load().nqs_local_energy(self._h, sp, B, _dev(e, torch.float64, "e_loc"),
                                       _MODES[mode], _stream()), "nqs_local_energy")
        return e

    def mcmc(self, spins, rand_bond, rand_u, accepted=None, mode: str = "auto"):
        """Metropolis steps of every chain (sample) of `spins`, in place:
        rand_bond [n_steps, B] int32 (its bits read as uint32) or int64 with
        values in [0, 2^31); rand_u FP64 [n_steps, B] in [0, 1).  Returns the
        per-chain accepted counts (int32 [B], added to)."""
        sp, B = self._spins(spins)
        if rand_bond.dim() != 2 or rand_bond.shape[1] != B or rand_u.shape != rand_bond.shape:
            raise ValueError("rand_bond and rand_u must both be [n_steps, B]")
        n_steps = rand_bond.shape[0]
        rb = rand_bond
        if rb.dtype != torch.int32:
            if bool(((rb < 0) | (rb >= 2 ** 31)).any()):
                raise ValueError("int64 rand_bond values must lie in [0, 2^31)")
            rb = rb.to(torch.int32)
        rb = rb.contiguous()
        ru = rand_u.to(torch.float64).contiguous()
        acc = accepted if accepted is not None else torch.zeros(B, dtype=torch.int32,
                                                                device=spins.device)
        _check(load().nqs_mcmc(self._h, sp, B, n_steps, _dev(rb, torch.int32, "rand_bond"),
                               _dev(ru, torch.float64, "rand_u"), _dev(acc, torch.int32, "accepted"),
                               _MODES[mode], _stream()), "nqs_mcmc")
        return acc

    def energy_stats(self, e_loc, out=None):
        st = out if out is not None else torch.empty(2, dtype=torch.float64, device=e_loc.device)
        _check(load().nqs_energy_stats(self._h, _dev(e_loc, torch.float64, "e_loc"),
                                       e_loc.numel(), _dev(st, torch.float64, "stats"),
                                       _stream()), "nqs_energy_stats")
        return st

    def log_deriv(self, spins, dtype: str = "fp32", out=None):
        sp, B = self._spins(spins)
        tdt = torch.float32 if dtype == "fp32" else torch.float64
        O = out if out is not None else torch.empty(B, self.P, dtype=tdt, device=spins.device)
        _check(load().nqs_log_deriv(self._h, sp, B, _dev(O, tdt, "O"), _DTYPES[dtype],
                                    _stream()), "nqs_log_deriv")
        return O

    def sr_solve(self, O, e_loc, diag_shift: float = 1e-4, n_iter: int = 100, out=None,
                 stats=None):
        odt = FP32 if O.dtype == torch.float32 else FP64
        B = O.shape[0]
        if O.shape[1] != self.P or e_loc.numel() != B:
            raise ValueError("O must be [B, P] and e_loc [B]")
        x = out if out is not None else torch.empty(self.P, dtype=torch.float64, device=O.device)
        st = stats if stats is not None else torch.empty(4, dtype=torch.float64, device=O.device)
        _check(load().nqs_sr_solve(self._h, _dev(O, O.dtype, "O"), odt,
                                   _dev(e_loc, torch.float64, "e_loc"), B, diag_shift, n_iter,
                                   _dev(x, torch.float64, "dtheta"),
                                   _dev(st, torch.float64, "stats"), _stream()), "nqs_sr_solve")
        return x, st

    def sr_solve_noalloc(self, O, e_loc, diag_shift: float = 1e-4, n_iter: int = 100, *,
                         out, stats):
        """nqs_sr_solve_noalloc: the SR solve with its workspace in the library's
        fixed device array (no allocation anywhere: out and stats are
        caller-provided FP64 [P] and [4] device tensors)."""
        odt = {torch.float32: FP32, torch.float64: FP64}[O.dtype]
        B = O.shape[0]
        if O.dim() != 2 or O.shape[1] != self.P or e_loc.numel() != B:
            raise ValueError("O must be [B, P] and e_loc [B]")
        if out.numel() != self.P or stats.numel() < 4:
            raise ValueError("out must hold P values and stats 4")
        _check(load().nqs_sr_solve_noalloc(self._h, _dev(O, O.dtype, "O"), odt,
                                           _dev(e_loc, torch.float64, "e_loc"), B,
                                           float(diag_shift), int(n_iter),
                                           _dev(out, torch.float64, "dtheta"),
                                           _dev(stats, torch.float64, "stats"), _stream()),
               "nqs_sr_solve_noalloc")
        return out, stats

    def sr_solve_recompute(self, spins, e_loc, diag_shift: float = 1e-4, n_iter: int = 100,
                           dtype: str = "fp32", chunk_rows: int = 0, out=None, stats=None):
        """SR with O recomputed from the spins in chunks of chunk_rows samples
        (0: as many as fit in 2 GiB); equals sr_solve on log_deriv's O."""
        sp, B = self._spins(spins)
        if e_loc.numel() != B:
            raise ValueError("e_loc must have one entry per sample")
        x = out if out is not None else torch.empty(self.P, dtype=torch.float64,
                                                    device=spins.device)
        st = stats if stats is not None else torch.empty(4, dtype=torch.float64,
                                                         device=spins.device)
        _check(load().nqs_sr_solve_recompute(self._h, sp, _DTYPES[dtype],
                                             _dev(e_loc, torch.float64, "e_loc"), B,
                                             diag_shift, n_iter, chunk_rows,
                                             _dev(x, torch.float64, "dtheta"),
                                             _dev(st, torch.float64, "stats"), _stream()),
               "nqs_sr_solve_recompute")
        return x, st

    def capacity(self, B: int) -> int:
        nn = self.J1 != 0 or (self.model == "tj" and self.t != 0)
        per = 2 * self.L * self.L * ((1 if nn else 0) + (1 if self.J2 != 0 else 0))
        return per * B

    def connected(self, spins):
        sp, B = self._spins(spins)
        dev = spins.device
        cap = max(self.capacity(B), 1)
        counts = torch.empty(max(B, 1), dtype=torch.int32, device=dev)
        offs = torch.empty(B + 1, dtype=torch.int64, device=dev)
        bonds = torch.empty(cap, dtype=torch.int32, device=dev)
        mu = torch.empty(cap, dtype=torch.int8, device=dev)
        ed = torch.empty(max(B, 1), dtype=torch.float64, device=dev)
        _check(load().nqs_connected(self._h, sp, B, ctypes.c_void_p(counts.data_ptr()),
                                    ctypes.c_void_p(offs.data_ptr()),
                                    ctypes.c_void_p(bonds.data_ptr()),
                                    ctypes.c_void_p(mu.data_ptr()), cap,
                                    ctypes.c_void_p(ed.data_ptr()), _stream()), "nqs_connected")
        return counts[:B], offs, bonds, mu, ed[:B]

    def log_ratios(self, spins, mode: str = "auto"):
        sp, B = self._spins(spins)
        cap = max(self.capacity(B), 1)
        d = torch.empty(cap, dtype=torch.float64, device=spins.device)
        _check(load().nqs_log_ratios(self._h, sp, B, _MODES[mode], _dev(d, torch.float64, "dlog"),
                                     cap, _stream()), "nqs_log_ratios")
        return d

    def get_error(self) -> int:
        v = ctypes.c_int32()
        _check(load().nqs_get_error(self._h, ctypes.byref(v)), "nqs_get_error")
        return v.value

    def enable_timing(self, on: bool = True):
        _check(load().nqs_enable_timing(self._h, 1 if on else 0), "nqs_enable_timing")

    def kernel_time(self):
        ms, n = ctypes.c_double(), ctypes.c_int64()
        _check(load().nqs_kernel_time(self._h, ctypes.byref(ms), ctypes.byref(n)),
               "nqs_kernel_time")
        return ms.value, n.value


def local_energy_multi(jobs, mode: str = "auto"):
    """jobs: list of (Context, spins tensor, e_loc tensor)."""
    arr = (ElocJob * len(jobs))()
    for i, (ctx, spins, e) in enumerate(jobs):
        sp, B = ctx._spins(spins)
        arr[i] = ElocJob(ctx.handle.value, sp.value, B, _dev(e, torch.float64, "e_loc").value)
    _check(load().nqs_local_energy_multi(arr, len(jobs), _MODES[mode], _stream()),
           "nqs_local_energy_multi")


def mfma_rate(kind: str = "bf16", workgroups: int = 4096, iters: int = 4000):
    """Sustained matrix-core rate of a register-only MFMA loop (nqs_mfma_rate):
    (launch ms, TFLOP/s); kind "bf16" (16x16x32) or "fp64" (16x16x4)."""
    ms, tf = ctypes.c_double(), ctypes.c_double()
    _check(load().nqs_mfma_rate({"bf16": 0, "fp64": 1}[kind], workgroups, iters,
                                ctypes.byref(ms), ctypes.byref(tf), _stream()), "nqs_mfma_rate")
    return ms.value, tf.value


def tune_key(L: int, K: int, C: int, dtype: str, J2: float) -> str:
    """Tune-cache key of a configuration (host only)."""
    buf = ctypes.create_string_buffer(128)
    _check(load().nqs_tune_key(L, K, C, _DTYPES[dtype], J2, buf, len(buf)), "nqs_tune_key")
    return buf.value.decode()


def tune_lookup(path: str, key: str):
    """The tune-cache entry of key in the file at path, or None (missing file or
    key, malformed file).  Host only."""
    m, nw, mt = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
    ci, cw = ctypes.c_int32(), ctypes.c_int32()
    code = load().nqs_tune_lookup(path.encode(), key.encode(), ctypes.byref(m), ctypes.byref(nw),
                                  ctypes.byref(mt), ctypes.byref(ci), ctypes.byref(cw))
    if code != 0:
        return None
    return {"mode": {v: k for k, v in _MODES.items()}[m.value], "full_nw": nw.value,
            "full_maxt": mt.value, "cone_items": ci.value, "cone_waves": cw.value}


class LogPsiFn(torch.autograd.Function):
    """log|psi(s)| as a differentiable function of the weights.

    forward: the weights set on the device from theta (nqs_set_weights_device:
    no host round trip, no synchronisation), then nqs_log_psi; backward: the
    same weights set again (the context may have been used with others in
    between), per-sample O = d log|psi| / d theta from the hand-written
    backward kernels (nqs_log_deriv, FP64), contracted with the incoming
    gradient."""

    @staticmethod
    def forward(ctx_, theta, spins, nctx):
        th = theta.detach().to(device=spins.device, dtype=torch.float64).contiguous()
        nctx.set_weights_device(th)
        la = nctx.log_psi(spins, with_sign=False)
        ctx_.save_for_backward(spins, th)
        ctx_.nctx = nctx
        ctx_.theta_device = theta.device
        return la

    @staticmethod
    def backward(ctx_, g):
        spins, th = ctx_.saved_tensors
        ctx_.nctx.set_weights_device(th)
        O = ctx_.nctx.log_deriv(spins, dtype="fp64")
        return (g.to(O.device, torch.float64) @ O).to(ctx_.theta_device), None, None
