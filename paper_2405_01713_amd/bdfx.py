"""Thin Python binding of the bdfx C ABI (include/bdfx.h).

The functions ``bdfx_*`` below carry the C names and only marshal arguments
(device pointers are passed as integers, e.g. ``tensor.data_ptr()``).  The
``Integrator`` helper owns torch tensors for the caller-owned device buffers
and forwards every step to the library: no part of the integration runs in
Python or PyTorch.  Importing this module does not need a GPU; calling the
library does, and it fails loudly when ``libbdfx.so`` is missing.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libbdfx.so")

BDFX_OK = 0
BDFX_EINVAL, BDFX_EWORKSPACE, BDFX_EHIP, BDFX_EORDER, BDFX_EUNSUPPORTED = -1, -2, -3, -4, -5
BDFX_CELL_RECORD_FULL = -10
BDFX_SCHED_STATIC = 0
BDFX_SCHED_QUEUE = 1
BDFX_SCHED_FUSED = 2
BDFX_JAC_ANALYTIC, BDFX_JAC_DQ = 0, 1
BDFX_GMRES_MAXL = 10
BDFX_MAX_LOCKSTEP = 16
MAX_SPECIES = 64

CELL_STATUS = {0: "success", -1: "too_much_work", -3: "err_failure", -4: "conv_failure",
               -6: "setup_failure", -9: "nonfinite", -10: "record_full"}

EXPORTED = ["bdfx_create", "bdfx_set_stream", "bdfx_destroy", "bdfx_last_error",
            "bdfx_mech_create", "bdfx_mech_destroy", "bdfx_mech_set_weights", "bdfx_mech_set_lnA",
            "bdfx_plan",
            "bdfx_bind", "bdfx_integrate", "bdfx_perturb", "bdfx_stats_summary",
            "bdfx_adjoint", "bdfx_autotune", "bdfx_set_tuning", "bdfx_get_tuning", "bdfx_typical_atol",
            "bdfx_get_record_layout", "bdfx_version", "bdfx_typical_atol_static"]


class MechDesc(C.Structure):
    _fields_ = [("n_species", C.c_int32), ("n_reactions", C.c_int32),
                ("reac", C.c_void_p), ("prod", C.c_void_p), ("lnA", C.c_void_p),
                ("EaR", C.c_void_p), ("lnK", C.c_void_p), ("cv", C.c_void_p),
                ("u0", C.c_void_p)]


class Options(C.Structure):
    _fields_ = [("rtol", C.c_double), ("atol", C.c_void_p), ("atol_len", C.c_int32),
                ("max_order", C.c_int32), ("max_steps", C.c_int32),
                ("lu_precision", C.c_int32), ("scheduler", C.c_int32),
                ("record_steps", C.c_int32), ("waves_per_block", C.c_int32),
                ("blocks_per_cu", C.c_int32), ("queue_chunk", C.c_int32),
                ("waves_per_simd", C.c_int32), ("cells_per_wave", C.c_int32),
                ("jacobian", C.c_int32), ("gmres_maxl", C.c_int32), ("lockstep", C.c_int32),
                ("max_err_test_fails", C.c_int32), ("max_conv_fails", C.c_int32),
                ("checkpoint_every", C.c_int32)]


class Summary(C.Structure):
    _fields_ = [("n_cells", C.c_int64), ("n_success", C.c_int64), ("n_failed", C.c_int64),
                ("nst", C.c_int64), ("nfe", C.c_int64), ("nni", C.c_int64),
                ("nsetups", C.c_int64), ("netf", C.c_int64), ("ncfn", C.c_int64),
                ("max_nst", C.c_int64), ("status_count", C.c_int64 * 11),
                ("nli", C.c_int64), ("ncfl", C.c_int64)]


class RecordLayout(C.Structure):
    _fields_ = [("cap", C.c_int32), ("stride", C.c_int32), ("off_steps", C.c_size_t),
                ("off_count", C.c_size_t), ("off_hpad", C.c_size_t), ("off_y0", C.c_size_t)]


class Tuning(C.Structure):
    _fields_ = [("mech", C.c_int32), ("waves_per_simd", C.c_int32),
                ("waves_per_block", C.c_int32), ("queue_chunk", C.c_int32),
                ("sample_cells", C.c_int64), ("ms", C.c_float), ("cells_per_wave", C.c_int32),
                ("tables", C.c_int32), ("fused", C.c_int32)]


STATS_DTYPE = np.dtype([("status", np.int32), ("nst", np.int32), ("nfe", np.int32),
                        ("nni", np.int32), ("nsetups", np.int32), ("netf", np.int32),
                        ("ncfn", np.int32), ("q_last", np.int32),
                        ("nli", np.int32), ("ncfl", np.int32),
                        ("h_last", np.float64), ("t_reached", np.float64)])
assert STATS_DTYPE.itemsize == 56

_lib = None


def lib():
    """Load libbdfx.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: run __graft_entry__.build() first")
        L = C.CDLL(LIB_PATH)
        P, I32, I64 = C.c_void_p, C.c_int32, C.c_int64
        sig = {
            "bdfx_create": ([C.POINTER(P), C.c_int, P], C.c_int),
            "bdfx_set_stream": ([P, P], C.c_int),
            "bdfx_destroy": ([P], C.c_int),
            "bdfx_last_error": ([P], C.c_char_p),
            "bdfx_mech_create": ([P, C.POINTER(MechDesc), C.POINTER(P)], C.c_int),
            "bdfx_mech_destroy": ([P], C.c_int),
            "bdfx_mech_set_weights": ([P, P], C.c_int),
            "bdfx_mech_set_lnA": ([P, P], C.c_int),
            "bdfx_plan": ([P, I64, I32, P, C.POINTER(Options), C.POINTER(C.c_size_t)], C.c_int),
            "bdfx_bind": ([P, P, C.c_size_t, P, I32, P, P, P, I32, P, P, P], C.c_int),
            "bdfx_integrate": ([P, C.c_double, C.c_double], C.c_int),
            "bdfx_perturb": ([P, C.c_uint64, I64, C.c_double], C.c_int),
            "bdfx_stats_summary": ([P, C.POINTER(Summary)], C.c_int),
            "bdfx_adjoint": ([P, P, P, P], C.c_int),
            "bdfx_autotune": ([P, C.c_double, C.c_double, I64, C.POINTER(Tuning)], C.c_int),
            "bdfx_set_tuning": ([P, C.POINTER(Tuning), I32], C.c_int),
            "bdfx_get_tuning": ([P, C.POINTER(Tuning), I32], C.c_int),
            "bdfx_typical_atol": ([P, C.c_double, P], C.c_int),
            "bdfx_typical_atol_static": ([C.c_int, P, P, I64, I32, I32, C.c_double, P, P], C.c_int),
            "bdfx_get_record_layout": ([P, C.POINTER(RecordLayout)], C.c_int),
            "bdfx_version": ([], C.c_char_p),
        }
        for name, (args, res) in sig.items():
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = res
        _lib = L
    return _lib


class BdfxError(RuntimeError):
    pass


def _check(rc, ctx=None):
    if rc != BDFX_OK:
        msg = lib().bdfx_last_error(ctx)
        raise BdfxError(f"bdfx error {rc}: {msg.decode() if msg else ''}")


# --- C-named entry points (argument marshalling only) ---------------------

def bdfx_version() -> str:
    return lib().bdfx_version().decode()


def bdfx_create(device: int = 0, stream: int = 0):
    h = C.c_void_p()
    _check(lib().bdfx_create(C.byref(h), int(device), C.c_void_p(stream)))
    return h


def bdfx_set_stream(ctx, stream: int):
    _check(lib().bdfx_set_stream(ctx, C.c_void_p(stream)), ctx)


def bdfx_destroy(ctx):
    _check(lib().bdfx_destroy(ctx))


def bdfx_last_error(ctx=None) -> str:
    m = lib().bdfx_last_error(ctx)
    return m.decode() if m else ""


def bdfx_mech_create(ctx, mech: dict):
    """mech: dict with n_species, n_reactions, reac/prod [R,3], lnA, EaR, lnK,
    and for a non-isothermal mechanism cv, u0 [S]."""
    f64 = lambda k: (None if mech.get(k) is None
                     else np.ascontiguousarray(mech[k], dtype=np.float64))
    keep = dict(
        reac=np.ascontiguousarray(mech["reac"], dtype=np.int32),
        prod=np.ascontiguousarray(mech["prod"], dtype=np.int32),
        lnA=np.ascontiguousarray(mech["lnA"], dtype=np.float64),
        EaR=None if mech.get("EaR") is None else np.ascontiguousarray(mech["EaR"], dtype=np.float64),
        lnK=None if mech.get("lnK") is None else np.ascontiguousarray(mech["lnK"], dtype=np.float64),
        cv=f64("cv"),
        u0=f64("u0"),
    )
    p = lambda a: None if a is None else a.ctypes.data_as(C.c_void_p)
    d = MechDesc(int(mech["n_species"]), int(mech["n_reactions"]), p(keep["reac"]),
                 p(keep["prod"]), p(keep["lnA"]), p(keep["EaR"]), p(keep["lnK"]), p(keep["cv"]),
                 p(keep["u0"]))
    h = C.c_void_p()
    _check(lib().bdfx_mech_create(ctx, C.byref(d), C.byref(h)), ctx)
    if mech.get("w") is not None:
        w = np.ascontiguousarray(mech["w"], dtype=np.float64)
        _check(lib().bdfx_mech_set_weights(h, w.ctypes.data_as(C.c_void_p)), ctx)
    return h


def bdfx_mech_destroy(mech):
    _check(lib().bdfx_mech_destroy(mech))


def bdfx_mech_set_lnA(mech, lnA_ptr, ctx=None):
    """Device-to-device copy of R doubles at lnA_ptr into the mechanism's lnA."""
    _check(lib().bdfx_mech_set_lnA(mech, C.c_void_p(int(lnA_ptr))), ctx)


def make_options(rtol, atol, max_order=5, max_steps=5000, lu_precision=64,
                 scheduler=BDFX_SCHED_STATIC, record_steps=0, waves_per_block=0,
                 blocks_per_cu=0, queue_chunk=0, waves_per_simd=0, cells_per_wave=0,
                 jacobian=0, gmres_maxl=0, lockstep=0, max_err_test_fails=0, max_conv_fails=0,
                 checkpoint_every=0):
    atol_arr = np.ascontiguousarray(np.atleast_1d(np.asarray(atol, dtype=np.float64)))
    o = Options(float(rtol), atol_arr.ctypes.data_as(C.c_void_p), int(atol_arr.size),
                int(max_order), int(max_steps), int(lu_precision), int(scheduler),
                int(record_steps), int(waves_per_block), int(blocks_per_cu), int(queue_chunk),
                int(waves_per_simd), int(cells_per_wave), int(jacobian), int(gmres_maxl),
                int(lockstep), int(max_err_test_fails), int(max_conv_fails),
                int(checkpoint_every))
    o._keep = atol_arr
    return o


def bdfx_plan(ctx, n_cells: int, mechs, opts: Options) -> int:
    arr = (C.c_void_p * len(mechs))(*[m.value for m in mechs])
    nbytes = C.c_size_t(0)
    _check(lib().bdfx_plan(ctx, int(n_cells), len(mechs), C.cast(arr, C.c_void_p),
                           C.byref(opts), C.byref(nbytes)), ctx)
    return int(nbytes.value)


def bdfx_bind(ctx, ws_ptr, ws_bytes, y_ptr, ldy, cell_mech_ptr, T_ptr, kscale_ptr, ldk,
              forcing_ptr, status_ptr, stats_ptr):
    v = lambda x: C.c_void_p(int(x) if x else 0)
    _check(lib().bdfx_bind(ctx, v(ws_ptr), C.c_size_t(int(ws_bytes)), v(y_ptr), int(ldy),
                           v(cell_mech_ptr), v(T_ptr), v(kscale_ptr), int(ldk), v(forcing_ptr),
                           v(status_ptr), v(stats_ptr)), ctx)


def bdfx_integrate(ctx, t0: float, t_out: float):
    _check(lib().bdfx_integrate(ctx, float(t0), float(t_out)), ctx)


def bdfx_perturb(ctx, seed: int, outer_step: int, amplitude: float):
    _check(lib().bdfx_perturb(ctx, C.c_uint64(int(seed)), int(outer_step), float(amplitude)), ctx)


def bdfx_typical_atol(ctx, eta: float, d_typical=None):
    _check(lib().bdfx_typical_atol(ctx, float(eta), d_typical), ctx)


def bdfx_typical_atol_static(device: int, stream: int, y_ptr: int, n_cells: int, ldy: int,
                             n_species: int, eta: float, atol_ptr: int, typical_ptr=None):
    """Allocation-free typical-value tolerances (no context); device pointers
    as integers."""
    _check(lib().bdfx_typical_atol_static(int(device), stream or None, y_ptr, int(n_cells),
                                          int(ldy), int(n_species), float(eta), atol_ptr,
                                          typical_ptr))


def bdfx_stats_summary(ctx) -> dict:
    s = Summary()
    _check(lib().bdfx_stats_summary(ctx, C.byref(s)), ctx)
    out = {k: getattr(s, k) for k, _ in Summary._fields_ if k != "status_count"}
    out["status_count"] = list(s.status_count)
    return out


def bdfx_adjoint(ctx, ybar_ptr, y0bar_ptr, lnA_bar_ptr):
    v = lambda x: C.c_void_p(int(x) if x else 0)
    _check(lib().bdfx_adjoint(ctx, v(ybar_ptr), v(y0bar_ptr), v(lnA_bar_ptr)), ctx)


def bdfx_get_record_layout(ctx) -> dict:
    r = RecordLayout()
    _check(lib().bdfx_get_record_layout(ctx, C.byref(r)), ctx)
    return {k: getattr(r, k) for k, _ in RecordLayout._fields_}


_TUNING_KEYS = ("mech", "waves_per_simd", "waves_per_block", "queue_chunk", "cells_per_wave",
                "sample_cells", "ms", "tables", "fused")


def bdfx_autotune(ctx, n_mech: int, t0: float, t_out: float, sample_cells: int = 0) -> list:
    out = (Tuning * max(n_mech, 1))()
    _check(lib().bdfx_autotune(ctx, float(t0), float(t_out), int(sample_cells), out), ctx)
    return [{k: getattr(t, k) for k in _TUNING_KEYS} for t in out[:n_mech]]


def bdfx_get_tuning(ctx, n_mech: int) -> list:
    out = (Tuning * max(n_mech, 1))()
    _check(lib().bdfx_get_tuning(ctx, out, n_mech), ctx)
    return [{k: getattr(t, k) for k in _TUNING_KEYS} for t in out[:n_mech]]


def bdfx_set_tuning(ctx, tunings: list):
    arr = (Tuning * max(len(tunings), 1))()
    for i, t in enumerate(tunings):
        for k in ("mech", "waves_per_simd", "waves_per_block", "queue_chunk", "cells_per_wave"):
            setattr(arr[i], k, int(t.get(k, 1) if k == "cells_per_wave" else t[k]))
    _check(lib().bdfx_set_tuning(ctx, arr, len(tunings)), ctx)


# --- convenience wrapper over torch device memory -------------------------

class Integrator:
    """Batch of cells on one GPU: owns the device tensors, calls the C ABI.

    ``mechs``: list of mechanism dicts; ``y0`` [N, S_max] float64; optional
    ``T`` [N], ``kscale`` [N, R_max], ``forcing`` [N, S_max], ``cell_mech`` [N].
    """

    def __init__(self, mechs, y0, rtol, atol, T=None, kscale=None, forcing=None, cell_mech=None,
                 device=0, stream=None, **opts):
        import torch

        if isinstance(mechs, dict):
            mechs = [mechs]
        self.torch = torch
        self.dev = torch.device("cuda", device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.dev)
        self.ctx = bdfx_create(device, self.stream.cuda_stream)
        self.mech_handles = [bdfx_mech_create(self.ctx, m) for m in mechs]
        self.mechs = mechs
        # state entries per cell (a non-isothermal mechanism adds the temperature)
        self.S_max = max(int(m["n_species"]) + (m.get("cv") is not None) for m in mechs)
        self.N, self.ldy = tuple(y0.shape)
        self.opts = make_options(rtol, atol, **opts)
        ws = bdfx_plan(self.ctx, self.N, self.mech_handles, self.opts)
        def t(a, dt):
            if a is None:
                return None
            if isinstance(a, torch.Tensor):
                return a.detach().to(device=self.dev, dtype=dt).contiguous().clone()
            return torch.as_tensor(np.ascontiguousarray(a), dtype=dt, device=self.dev)
        self.y = t(y0, torch.float64)
        self.T = t(T, torch.float64)
        self.kscale = t(kscale, torch.float64)
        self.forcing = t(forcing, torch.float64)
        self.cell_mech = t(cell_mech, torch.int32)
        self.status = torch.zeros(self.N, dtype=torch.int32, device=self.dev)
        self.stats = torch.zeros(self.N * STATS_DTYPE.itemsize, dtype=torch.uint8, device=self.dev)
        self.ws = torch.empty(max(ws, 256), dtype=torch.uint8, device=self.dev)
        self.ws_bytes = ws
        ptr = lambda x: 0 if x is None else x.data_ptr()
        self.ldk = 0 if kscale is None else int(np.shape(kscale)[1])
        bdfx_bind(self.ctx, ptr(self.ws), self.ws.numel(), ptr(self.y), self.ldy,
                  ptr(self.cell_mech), ptr(self.T), ptr(self.kscale), self.ldk, ptr(self.forcing),
                  ptr(self.status), ptr(self.stats))

    def integrate(self, t0, t_out):
        bdfx_integrate(self.ctx, t0, t_out)

    def perturb(self, seed, outer_step, amplitude):
        bdfx_perturb(self.ctx, seed, outer_step, amplitude)

    def typical_atol(self, eta, typical=None):
        """Typical-value tolerances from the current states (bdfx_typical_atol);
        ``typical``: optional float64 device tensor [n_mech, S_max] that
        receives the typical values.  eta = 0 returns to the options' atol."""
        if typical is not None:
            assert typical.is_cuda and typical.dtype == self.torch.float64
            assert typical.is_contiguous() and typical.numel() >= len(self.mechs) * self.S_max
        bdfx_typical_atol(self.ctx, eta, None if typical is None else typical.data_ptr())

    def set_lnA(self, lnA, mech=0):
        """New ln pre-exponential factors for mechanism ``mech`` from a float64
        device tensor [R] (a device copy enqueued on the context's stream)."""
        torch = self.torch
        R = int(self.mechs[mech]["n_reactions"])
        a = lnA.detach().to(device=self.dev, dtype=torch.float64).contiguous()
        assert a.numel() == R
        bdfx_mech_set_lnA(self.mech_handles[mech], a.data_ptr(), self.ctx)
        self._keep_lnA = a

    def set_state(self, y0):
        self.y.copy_(self.torch.as_tensor(np.ascontiguousarray(y0), dtype=self.torch.float64))

    def summary(self):
        return bdfx_stats_summary(self.ctx)

    def adjoint(self, ybar):
        """Discrete adjoint of the last integrate (needs record_steps > 0).
        Returns (dL/dy0 [N, ldy], dL/dlnA [n_mech, R_max]) as device tensors."""
        torch = self.torch
        yb = (ybar.detach() if isinstance(ybar, torch.Tensor) else torch.as_tensor(np.asarray(ybar)))
        yb = yb.to(device=self.dev, dtype=torch.float64).contiguous()
        y0bar = torch.zeros_like(self.y)
        R_max = max(int(m["n_reactions"]) for m in self.mechs)
        lnA_bar = torch.zeros((len(self.mechs), R_max), dtype=torch.float64, device=self.dev)
        bdfx_adjoint(self.ctx, yb.data_ptr(), y0bar.data_ptr(), lnA_bar.data_ptr())
        self._keep = yb
        return y0bar, lnA_bar

    def step_record(self, cells):
        """The recorded accepted steps of the given cells after an integrate
        with record_steps > 0 (bdfx_get_record_layout): a list of dicts with
        n, h_pad, y [n][S], h [n], q [n], rebuild [n] and y0 [S], S the
        cell's state length (host copies; synchronises)."""
        torch = self.torch
        lay = bdfx_get_record_layout(self.ctx)
        cap, stride = lay["cap"], lay["stride"]
        torch.cuda.synchronize(self.dev)
        f64 = lambda off, count: self.ws[off:off + 8 * count].view(torch.float64)
        count = self.ws[lay["off_count"]:lay["off_count"] + 4 * self.N].view(torch.int32).cpu().numpy()
        hpad = f64(lay["off_hpad"], self.N).cpu().numpy()
        cm = (np.zeros(self.N, dtype=np.int64) if self.cell_mech is None
              else self.cell_mech.cpu().numpy())
        out = []
        for c in np.atleast_1d(cells):
            c = int(c)
            m = self.mechs[int(cm[c])]
            S = int(m["n_species"]) + (m.get("cv") is not None)
            n = int(count[c])
            steps = f64(lay["off_steps"] + 8 * c * cap * stride, cap * stride).view(cap, stride)
            steps = steps[:n].cpu().numpy()
            code = steps[:, S + 1].astype(np.int64)
            y0 = f64(lay["off_y0"] + 8 * c * stride, stride).cpu().numpy()[:S]
            out.append(dict(n=n, h_pad=float(hpad[c]), y=steps[:, :S].copy(), h=steps[:, S].copy(),
                            q=(code & 255).astype(np.int32), rebuild=(code >> 8).astype(np.int32),
                            y0=y0))
        return out

    def autotune(self, t0, t_out, sample_cells=0, cache=None):
        """Pick the launch shape per mechanism with bdfx_autotune().  With
        ``cache`` (a JSON file path, one per machine) results are looked up by
        compute-unit count, mechanism size, LU precision, scheduler and
        linear solver, and stored after tuning."""
        import json

        # the cache file belongs to one machine; the key tells apart batch
        # shapes and GPUs of different size
        n_cu = self.torch.cuda.get_device_properties(self.dev).multi_processor_count
        key = lambda m: (f"CU{n_cu}|S{self.mechs[m]['n_species']}|R{self.mechs[m]['n_reactions']}"
                         f"{'|thermal' if self.mechs[m].get('cv') is not None else ''}"
                         f"|lu{self.opts.lu_precision}|sched{self.opts.scheduler}"
                         f"{'|dq' if self.opts.jacobian else ''}"
                         f"{f'|gmres{self.opts.gmres_maxl}' if self.opts.gmres_maxl else ''}"
                         f"{f'|lock{self.opts.lockstep}' if self.opts.lockstep else ''}")
        db = {}
        if cache and os.path.exists(cache):
            with open(cache) as fh:
                db = json.load(fh)
        hits = [dict(db[key(m)], mech=m) for m in range(len(self.mechs)) if key(m) in db]
        if cache and len(hits) == len(self.mechs):
            bdfx_set_tuning(self.ctx, hits)
            return hits
        res = bdfx_autotune(self.ctx, len(self.mechs), t0, t_out, sample_cells)
        if cache:
            for r in res:
                db[key(r["mech"])] = {k: r[k] for k in _TUNING_KEYS if k != "mech"}
            tmp = cache + ".tmp"
            with open(tmp, "w") as fh:
                json.dump(db, fh, indent=1, sort_keys=True)
            os.replace(tmp, cache)
        return res

    def tuning(self):
        """Launch shape in effect per mechanism (bdfx_get_tuning())."""
        return bdfx_get_tuning(self.ctx, len(self.mechs))

    def outer_loop(self, n_outer, dt, seed, amplitude, t0=0.0, typical_every=0, eta=1e-10):
        """Operator-splitting outer loop on the current stream: for k = 0 ..
        n_outer-1, perturb the states (outer step k of the counter-based
        perturbation, skipped when amplitude == 0), recompute the
        typical-value tolerances every ``typical_every`` outer steps (k = 0,
        K, 2K, ...; 0 = never), then integrate over [t0 + k dt, t0 + (k+1) dt]."""
        for k in range(n_outer):
            if amplitude != 0.0:
                self.perturb(seed, k, amplitude)
            if typical_every > 0 and k % typical_every == 0:
                self.typical_atol(eta)
            self.integrate(t0 + k * dt, t0 + (k + 1) * dt)

    def capture_outer_loop(self, n_outer, dt, seed, amplitude, t0=0.0, typical_every=0,
                           eta=1e-10):
        """Capture outer_loop() in a HIP graph (torch.cuda.CUDAGraph).

        The graph holds only the library's kernels (perturbation, queue reset
        by a fill kernel, integrator launches) with the bound buffers; replay
        it with ``g.replay()`` on any stream.  The context's stream is switched
        to a side stream for the capture and restored afterwards."""
        torch = self.torch
        side = torch.cuda.Stream(device=self.dev)
        side.wait_stream(self.stream)
        g = torch.cuda.CUDAGraph()
        bdfx_set_stream(self.ctx, side.cuda_stream)
        try:
            with torch.cuda.graph(g, stream=side):
                self.outer_loop(n_outer, dt, seed, amplitude, t0, typical_every, eta)
        finally:
            bdfx_set_stream(self.ctx, self.stream.cuda_stream)
        self.stream.wait_stream(side)
        return g

    def cell_stats(self) -> np.ndarray:
        return self.stats.cpu().numpy().view(STATS_DTYPE)

    def state(self) -> np.ndarray:
        return self.y.cpu().numpy()

    def close(self):
        if self.ctx:
            self.torch.cuda.synchronize(self.dev)
            for m in self.mech_handles:
                bdfx_mech_destroy(m)
            bdfx_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def make_bdf_function():
    """torch.autograd.Function over the library: forward integrates with step
    recording, backward runs the discrete adjoint (bdfx_adjoint).

    One bound Integrator per batch shape, mechanism structure, tolerances and
    device is created on first use and reused: each forward copies y0, T and
    lnA into it on the device and enqueues the integration, with no new
    context, workspace or host synchronisation.  A cell that fails (negative
    status) returns NaN in place of y(t_out), and its gradients are NaN (the
    lnA gradient, a sum over cells, is NaN if any cell failed).  One
    forward/backward pair may be in flight per cached Integrator: a backward
    whose forward was overwritten by a later forward raises."""
    import torch

    cache = {}

    def key_of(y0, mech, T, rtol, atol, record_steps):
        parts = [tuple(y0.shape), str(y0.device), int(mech["n_species"]),
                 int(mech["n_reactions"]), T is None, float(rtol),
                 np.asarray(atol, dtype=np.float64).tobytes(), int(record_steps)]
        for k in ("reac", "prod", "EaR", "lnK"):
            v = mech.get(k)
            parts.append(None if v is None else np.ascontiguousarray(v).tobytes())
        return tuple(parts)

    class BDFFunction(torch.autograd.Function):
        @staticmethod
        def forward(ctx, y0, lnA, mech, T, t_out, rtol, atol, record_steps=4096):
            k = key_of(y0, mech, T, rtol, atol, record_steps)
            integ = cache.get(k)
            if integ is None:
                m = dict(mech)
                m["lnA"] = np.asarray(mech["lnA"], dtype=np.float64)
                integ = Integrator([m], y0, rtol, atol, T=T, device=y0.device.index or 0,
                                   record_steps=record_steps)
                integ.generation = 0
                cache[k] = integ
            integ.y.copy_(y0.detach())
            if T is not None:
                integ.T.copy_(torch.as_tensor(T, dtype=torch.float64, device=integ.dev))
            integ.set_lnA(lnA)
            integ.integrate(0.0, float(t_out))
            integ.generation += 1
            ctx.integ, ctx.generation = integ, integ.generation
            failed = integ.status != 0
            ctx.failed = failed.clone()
            return torch.where(failed[:, None], torch.full_like(integ.y, float("nan")), integ.y)

        @staticmethod
        def backward(ctx, ybar):
            integ = ctx.integ
            if integ.generation != ctx.generation:
                raise RuntimeError("BDFFunction: a later forward on the same batch replaced the "
                                   "step record this backward needs")
            y0bar, lnA_bar = integ.adjoint(ybar)
            R = int(integ.mechs[0]["n_reactions"])
            nan = float("nan")
            failed = ctx.failed
            y0bar = torch.where(failed[:, None], torch.full_like(y0bar, nan), y0bar)
            g = lnA_bar[0, :R].clone()
            g = torch.where(failed.any(), torch.full_like(g, nan), g)
            return y0bar, g, None, None, None, None, None, None

    BDFFunction.cache = cache
    return BDFFunction
