"""ctypes binding of the FP64 CPU oracle (``bdf_oracle.c``).

TEST INFRASTRUCTURE ONLY: imported by the test suite, the smoke check and the
benchmark's CPU-baseline leg.  It never imports the product package and the
product never imports it.  Inputs are plain numpy arrays (e.g. from the shared
seeded generators); outputs are numpy arrays.
"""
from __future__ import annotations

import contextlib
import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "bdf_oracle.c")
LIB = os.path.join(HERE, "liboracle.so")

QMAX = 5
SLOTS = 3

STATUS = {0: "success", -1: "too_much_work", -3: "err_failure", -4: "conv_failure",
          -6: "setup_failure", -9: "nonfinite", -10: "record_full"}


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (plain -O2, no fast-math, no FMA contraction)."""
    if force or not os.path.exists(LIB):
        cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off",
               "-Wall", "-o", LIB + ".tmp", SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(LIB + ".tmp", LIB)
    return LIB


class Mech(C.Structure):
    _fields_ = [("n_species", C.c_int32), ("n_reactions", C.c_int32),
                ("reac", C.c_void_p), ("prod", C.c_void_p),
                ("lnA", C.c_void_p), ("EaR", C.c_void_p), ("lnK", C.c_void_p),
                ("cv", C.c_void_p), ("u0", C.c_void_p)]


class Opts(C.Structure):
    _fields_ = [("rtol", C.c_double), ("atol", C.c_void_p), ("atol_len", C.c_int32),
                ("max_order", C.c_int32), ("max_steps", C.c_int32), ("jac_dq", C.c_int32),
                ("gmres_maxl", C.c_int32), ("max_netf", C.c_int32), ("max_ncf", C.c_int32)]


class Stats(C.Structure):
    _fields_ = [("status", C.c_int32), ("nst", C.c_int32), ("nfe", C.c_int32),
                ("nni", C.c_int32), ("nsetups", C.c_int32), ("netf", C.c_int32),
                ("ncfn", C.c_int32), ("q_last", C.c_int32),
                ("nli", C.c_int32), ("ncfl", C.c_int32),
                ("h_last", C.c_double), ("t_reached", C.c_double)]


STATS_DTYPE = np.dtype([("status", np.int32), ("nst", np.int32), ("nfe", np.int32),
                        ("nni", np.int32), ("nsetups", np.int32), ("netf", np.int32),
                        ("ncfn", np.int32), ("q_last", np.int32),
                        ("nli", np.int32), ("ncfl", np.int32),
                        ("h_last", np.float64), ("t_reached", np.float64)])
assert STATS_DTYPE.itemsize == C.sizeof(Stats) == 56


class Record(C.Structure):
    _fields_ = [("cap", C.c_int32), ("n", C.c_int32), ("h_pad", C.c_double),
                ("y", C.c_void_p), ("h", C.c_void_p), ("q", C.c_void_p),
                ("rebuild", C.c_void_p)]


_lib = None


def lib():
    """The oracle library: liboracle.so, built on first use, or the build named
    by the environment variable BDFX_ORACLE_LIB (e.g. a sanitizer build)."""
    global _lib
    if _lib is None:
        path = os.environ.get("BDFX_ORACLE_LIB")
        if not path:
            path = LIB
            if not os.path.exists(LIB):
                build()
        _lib = load(path)
    return _lib


@contextlib.contextmanager
def use_library(path):
    """Run the bindings against another build of the oracle (for example a
    copy with a deliberately planted mistake, to show that a pin detects it)."""
    global _lib
    saved = _lib
    _lib = load(path)
    try:
        yield _lib
    finally:
        _lib = saved


def load(path):
    """Open an oracle library and declare its functions."""
    if True:
        L = C.CDLL(path)
        P = C.c_void_p
        L.orc_rates.argtypes = [P, C.c_double, P, P, P]
        L.orc_rhs.argtypes = [P, P, P, P, P, P]
        L.orc_jac.argtypes = [P, P, P, P, P]
        L.orc_rhs_thermal.argtypes = [P, P, P, P, P]
        L.orc_jacobian_dq.argtypes = [P, C.c_double, P, P, P, P, C.c_double, P]
        L.orc_jac_thermal.argtypes = [P, P, P, P, P]
        L.orc_gmres_solve.argtypes = [P, C.c_double, P, P, P, P, C.c_double, C.c_int32,
                                      C.c_double, P, P, P, P]
        L.orc_gmres_solve.restype = C.c_int32
        L.orc_lu_factor.argtypes = [C.c_int, P, P]
        L.orc_lu_factor.restype = C.c_int32
        L.orc_lu_solve.argtypes = [C.c_int, P, P, P]
        L.orc_wrms.argtypes = [C.c_int, P, P]
        L.orc_wrms.restype = C.c_double
        L.orc_bdf_coeffs.argtypes = [C.c_int, P, P, P]
        L.orc_integrate_cell.argtypes = [P, P, C.c_double, P, P, C.c_double, C.c_double, P, P, P,
                                         P]
        L.orc_integrate_cell.restype = C.c_int32
        L.orc_integrate_batch.argtypes = [C.c_int64, P, P, P, P, P, C.c_int32, P, C.c_int32,
                                          C.c_double, C.c_double, P, P, C.c_int32]
        L.orc_max_threads.restype = C.c_int32
        L.orc_integrate_lockstep_batch.argtypes = [C.c_int64, C.c_int32, C.c_int32, P, P, P, P,
                                                   P, C.c_int32, P, C.c_int32, C.c_double,
                                                   C.c_double, P, P, C.c_int32]
        L.orc_fixed_steps.argtypes = [P, P, P, P, C.c_int, C.c_double, C.c_int, P]
        L.orc_fixed_steps.restype = C.c_int32
        L.orc_replay_cell.argtypes = [P, P, P, P, P, P, P, P]
        L.orc_replay_cell.restype = C.c_int32
        L.orc_tangent_cell.argtypes = [P, P, P, P, P, P, P, P, P, P]
        L.orc_tangent_cell.restype = C.c_int32
        L.orc_adjoint_cell.argtypes = [P, P, P, P, P, P, P, P, P, P]
        L.orc_adjoint_cell.restype = C.c_int32
        L.orc_splitmix64.argtypes = [C.c_uint64]
        L.orc_splitmix64.restype = C.c_uint64
        L.orc_perturb_uniform.argtypes = [C.c_uint64, C.c_int64, C.c_int64, C.c_int32]
        L.orc_perturb_uniform.restype = C.c_double
        L.orc_perturb_batch.argtypes = [C.c_int64, P, C.c_int32, P, P, C.c_uint64, C.c_int64,
                                        C.c_double]
        L.orc_perturb_cells.argtypes = [C.c_int64, P, P, C.c_int32, P, P, C.c_uint64,
                                        C.c_int64, C.c_double]
        L.orc_lte_lower.argtypes = [C.c_int, C.c_int, P, P]
        L.orc_lte_lower.restype = C.c_double
        L.orc_lte_higher.argtypes = [C.c_int, C.c_int, P, P, C.c_double, C.c_double, P]
        L.orc_lte_higher.restype = C.c_double
        L.orc_initial_step_cell.argtypes = [P, P, C.c_double, P, P, C.c_double, C.c_double, P, P]
        L.orc_initial_step_cell.restype = C.c_double
        L.orc_steps.argtypes = [P, P, P, P, C.c_int, C.c_int, P, P, P, P, P, P]
        L.orc_steps.restype = C.c_int32
        L.orc_set_threads.argtypes = [C.c_int32]
    return L


def _p(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def _f64(a):
    return None if a is None else np.ascontiguousarray(a, dtype=np.float64)


class OracleMech:
    """Holds contiguous copies of a mechanism dict and its C description."""

    def __init__(self, mech: dict):
        self.S = int(mech["n_species"])
        self.R = int(mech["n_reactions"])
        self.reac = np.ascontiguousarray(mech["reac"], dtype=np.int32)
        self.prod = np.ascontiguousarray(mech["prod"], dtype=np.int32)
        self.lnA = _f64(mech["lnA"])
        self.EaR = _f64(mech.get("EaR"))
        self.lnK = _f64(mech.get("lnK"))
        self.cv = _f64(mech.get("cv"))
        self.u0 = _f64(mech.get("u0"))
        self.thermal = self.cv is not None
        self.c = Mech(self.S, self.R, _p(self.reac), _p(self.prod), _p(self.lnA),
                      _p(self.EaR), _p(self.lnK), _p(self.cv), _p(self.u0))

    @property
    def ptr(self):
        return C.byref(self.c)


def _opts(rtol, atol, max_order=5, max_steps=5000, jac_dq=False, gmres_maxl=0, max_netf=0,
          max_ncf=0):
    atol_arr = np.atleast_1d(np.asarray(atol, dtype=np.float64)).copy()
    o = Opts(float(rtol), _p(atol_arr), int(atol_arr.size), int(max_order), int(max_steps),
             int(bool(jac_dq)), int(gmres_maxl), int(max_netf), int(max_ncf))
    return o, atol_arr


def rates(mech, T=1.0, kscale=None):
    m = OracleMech(mech)
    kf = np.zeros(m.R)
    kr = np.zeros(m.R)
    ks = _f64(kscale)
    lib().orc_rates(m.ptr, float(T), _p(ks), _p(kf), _p(kr))
    return kf, kr


def rhs(mech, kf, kr, y, F=None):
    m = OracleMech(mech)
    kf, kr, y, F = _f64(kf), _f64(kr), _f64(y), _f64(F)
    f = np.zeros(m.S)
    lib().orc_rhs(m.ptr, _p(kf), _p(kr), _p(F), _p(y), _p(f))
    return f


def rhs_thermal(mech, x, kscale=None, F=None):
    """Non-isothermal right-hand side: x = (y_0 .. y_{S-1}, T)."""
    m = OracleMech(mech)
    x = _f64(x)
    f = np.zeros(m.S + 1)
    lib().orc_rhs_thermal(m.ptr, _p(_f64(kscale)), _p(_f64(F)), _p(x), _p(f))
    return f


def jac_thermal(mech, x, kscale=None, F=None):
    """Analytic (S+1) x (S+1) Jacobian of rhs_thermal."""
    m = OracleMech(mech)
    x = _f64(x)
    J = np.zeros((m.S + 1, m.S + 1))
    lib().orc_jac_thermal(m.ptr, _p(_f64(kscale)), _p(_f64(F)), _p(x), _p(J))
    return J


def jacobian_dq(mech, y, ewt, h, T=1.0, kscale=None, F=None):
    """Difference-quotient Jacobian (n x n, n = state length) at y."""
    m = OracleMech(mech)
    y = _f64(y)
    n = m.S + (1 if m.thermal else 0)
    J = np.zeros((n, n))
    lib().orc_jacobian_dq(m.ptr, float(T), _p(_f64(kscale)), _p(_f64(F)), _p(y), _p(_f64(ewt)),
                          float(h), _p(J))
    return J


def gmres_solve(mech, y, ewt, gamma, b, maxl=5, delta=0.0, T=1.0, kscale=None, F=None):
    """One matrix-free GMRES solve of (I - gamma J(y)) x = b on the system
    scaled by ewt.  Returns (x, code, iterations, residual norm of the scaled
    system); code 0 converged to delta, 1 reduced, 2 not reduced."""
    m = OracleMech(mech)
    y, ewt, b = _f64(y), _f64(ewt), _f64(b)
    x = np.zeros(y.size)
    nli = C.c_int32(0)
    rho = C.c_double(0.0)
    code = lib().orc_gmres_solve(m.ptr, float(T), _p(_f64(kscale)), _p(_f64(F)), _p(y), _p(ewt),
                                 float(gamma), int(maxl), float(delta), _p(b), _p(x),
                                 C.byref(nli), C.byref(rho))
    return x, int(code), int(nli.value), float(rho.value)


def jac(mech, kf, kr, y):
    m = OracleMech(mech)
    kf, kr, y = _f64(kf), _f64(kr), _f64(y)
    J = np.zeros((m.S, m.S))
    lib().orc_jac(m.ptr, _p(kf), _p(kr), _p(y), _p(J))
    return J


def lu_factor(A):
    A = np.array(A, dtype=np.float64, order="C")
    n = A.shape[0]
    perm = np.zeros(n, dtype=np.int32)
    info = lib().orc_lu_factor(n, _p(A), _p(perm))
    return A, perm, int(info)


def lu_solve(LU, perm, b):
    LU = _f64(LU)
    perm = np.ascontiguousarray(perm, dtype=np.int32)
    x = np.array(b, dtype=np.float64)
    lib().orc_lu_solve(LU.shape[0], _p(LU), _p(perm), _p(x))
    return x


def wrms(v, w):
    v, w = _f64(v), _f64(w)
    return float(lib().orc_wrms(v.size, _p(v), _p(w)))


def bdf_coeffs(q, xi):
    """xi: sequence xi_1..xi_{q+1}.  Returns (l[0..q], Cerr)."""
    x = np.zeros(QMAX + 2)
    x[1:q + 2] = np.asarray(xi, dtype=np.float64)[: q + 1]
    l = np.zeros(QMAX + 2)
    c = C.c_double(0.0)
    lib().orc_bdf_coeffs(int(q), _p(x), _p(l), C.byref(c))
    return l[: q + 1].copy(), c.value


def integrate(mechs, y0, t0, t_out, rtol, atol, T=None, kscale=None, F=None, cell_mech=None,
              max_order=5, max_steps=5000, nthreads=0, jac_dq=False, gmres_maxl=0, lockstep=0,
              max_netf=0, max_ncf=0):
    """Integrate a batch of cells; returns (y, stats structured array).
    jac_dq: Jacobian by difference quotients instead of the analytic one.
    gmres_maxl > 0: inexact Newton with matrix-free GMRES of that Krylov
    dimension (approaches 1A/1B) instead of the direct solve.
    lockstep = B > 0: the cells of each mechanism, in index order, are
    integrated in lock-step batches of B (one step size and one WRMS norm
    per batch; direct solver, analytic Jacobian).
    max_netf / max_ncf: error-test / Newton convergence failures in one step
    that fail a cell (0: the defaults 7 and 10)."""
    if isinstance(mechs, dict):
        mechs = [mechs]
    oms = [OracleMech(m) for m in mechs]
    arr = (Mech * len(oms))(*[m.c for m in oms])
    y = np.array(y0, dtype=np.float64, order="C", copy=True)
    N, ldy = y.shape
    T = _f64(T)
    ks = _f64(kscale)
    ldk = 0 if ks is None else ks.shape[1]
    F = _f64(F)
    cm = None if cell_mech is None else np.ascontiguousarray(cell_mech, dtype=np.int32)
    o, atol_arr = _opts(rtol, atol, max_order, max_steps, jac_dq, gmres_maxl, max_netf, max_ncf)
    stats = np.zeros(N, dtype=STATS_DTYPE)
    if lockstep:
        if not 1 <= lockstep <= 16 or jac_dq or gmres_maxl:
            raise ValueError("lock-step batches: 1..16 cells, direct solver, analytic Jacobian")
        lib().orc_integrate_lockstep_batch(N, int(lockstep), len(oms), C.cast(arr, C.c_void_p),
                                           _p(cm), C.byref(o), _p(T), _p(ks), ldk, _p(F), ldy,
                                           float(t0), float(t_out), _p(y), _p(stats),
                                           int(nthreads))
        return y, stats
    lib().orc_integrate_batch(N, C.cast(arr, C.c_void_p), _p(cm), C.byref(o), _p(T), _p(ks),
                              ldk, _p(F), ldy, float(t0), float(t_out), _p(y), _p(stats),
                              int(nthreads))
    return y, stats


def max_threads():
    return int(lib().orc_max_threads())


def integrate_record(mech, y0, t0, t_out, rtol, atol, T=1.0, kscale=None, F=None, max_order=5,
                     max_steps=5000, cap=20000):
    """One cell with the accepted-step record.  Returns (y, stats dict, record dict)."""
    m = OracleMech(mech)
    S = m.S
    y = np.array(y0, dtype=np.float64, copy=True)
    ks, F = _f64(kscale), _f64(F)
    o, atol_arr = _opts(rtol, atol, max_order, max_steps)
    ry = np.zeros((cap, S))
    rh = np.zeros(cap)
    rq = np.zeros(cap, dtype=np.int32)
    rb = np.zeros(cap, dtype=np.int32)
    rec = Record(cap, 0, 0.0, _p(ry), _p(rh), _p(rq), _p(rb))
    st = Stats()
    zout = np.zeros((QMAX + 1, S))
    lib().orc_integrate_cell(m.ptr, C.byref(o), float(T), _p(ks), _p(F), float(t0), float(t_out),
                             _p(y), C.byref(st), C.byref(rec), _p(zout))
    n = rec.n
    record = dict(n=n, h_pad=rec.h_pad, y=ry[:n].copy(), h=rh[:n].copy(), q=rq[:n].copy(),
                  rebuild=rb[:n].copy(), z_final=zout)
    stats = {k: getattr(st, k) for k, _ in Stats._fields_}
    return y, stats, record


def _crec(record, S):
    n = int(record["n"])
    cap = max(n, 1)
    ry = np.zeros((cap, S))
    ry[:n] = record["y"]
    rh = np.zeros(cap)
    rh[:n] = record["h"]
    rq = np.zeros(cap, dtype=np.int32)
    rq[:n] = record["q"]
    rb = np.zeros(cap, dtype=np.int32)
    rb[:n] = record["rebuild"]
    keep = (ry, rh, rq, rb)
    return Record(cap, n, float(record["h_pad"]), _p(ry), _p(rh), _p(rq), _p(rb)), keep


def replay(mech, kf, kr, y0, record, F=None):
    """Frozen replay with exact correctors.  Returns (y_out, replayed y_n [n][S])."""
    m = OracleMech(mech)
    S = m.S
    kf, kr, F, y0 = _f64(kf), _f64(kr), _f64(F), _f64(y0)
    rec, keep = _crec(record, S)
    yout = np.zeros(S)
    yrec = np.zeros((max(record["n"], 1), S))
    rc = lib().orc_replay_cell(m.ptr, _p(kf), _p(kr), _p(F), _p(y0), C.byref(rec), _p(yout),
                               _p(yrec))
    if rc:
        raise RuntimeError(f"replay failed: {rc}")
    return yout, yrec[: record["n"]]


def tangent(mech, kf, kr, y0, record, yrec, dy0, dp, F=None):
    m = OracleMech(mech)
    S = m.S
    kf, kr, F, y0 = _f64(kf), _f64(kr), _f64(F), _f64(y0)
    yr = np.zeros((max(record["n"], 1), S))
    yr[: record["n"]] = yrec
    rec, keep = _crec(record, S)
    dy0, dp = _f64(dy0), _f64(dp)
    out = np.zeros(S)
    rc = lib().orc_tangent_cell(m.ptr, _p(kf), _p(kr), _p(F), _p(y0), C.byref(rec), _p(yr),
                                _p(dy0), _p(dp), _p(out))
    if rc:
        raise RuntimeError(f"tangent failed: {rc}")
    return out


def adjoint(mech, kf, kr, y0, record, yrec, ybar, F=None):
    """Returns (y0bar [S], pbar [R]) for the frozen map along yrec."""
    m = OracleMech(mech)
    S = m.S
    kf, kr, F, y0 = _f64(kf), _f64(kr), _f64(F), _f64(y0)
    yr = np.zeros((max(record["n"], 1), S))
    yr[: record["n"]] = yrec
    rec, keep = _crec(record, S)
    ybar = _f64(ybar)
    y0bar = np.zeros(S)
    pbar = np.zeros(m.R)
    rc = lib().orc_adjoint_cell(m.ptr, _p(kf), _p(kr), _p(F), _p(y0), C.byref(rec), _p(yr),
                                _p(ybar), _p(y0bar), _p(pbar))
    if rc:
        raise RuntimeError(f"adjoint failed: {rc}")
    return y0bar, pbar


def fixed_steps(mech, kf, kr, z, q, h, nsteps, F=None):
    m = OracleMech(mech)
    kf, kr, F = _f64(kf), _f64(kr), _f64(F)
    zz = np.array(z, dtype=np.float64, order="C", copy=True)
    rc = lib().orc_fixed_steps(m.ptr, _p(kf), _p(kr), _p(F), int(q), float(h), int(nsteps),
                               _p(zz))
    if rc:
        raise RuntimeError(f"fixed_steps failed: {rc}")
    return zz


def lte_lower(q, zq, ewt):
    """Order-selection estimate of the local error of the order q-1 method from
    the top Nordsieck column z_q of the order-q array (WRMS norm, weights ewt)."""
    zq, ewt = _f64(zq), _f64(ewt)
    return float(lib().orc_lte_lower(zq.size, int(q), _p(zq), _p(ewt)))


def lte_higher(q, e, eprev, h, hprev, ewt):
    """Order-selection estimate of the local error of the order q+1 method from
    the corrections e (step of size h) and eprev (previous step, size hprev)."""
    e, eprev, ewt = _f64(e), _f64(eprev), _f64(ewt)
    return float(lib().orc_lte_higher(e.size, int(q), _p(e), _p(eprev), float(h), float(hprev),
                                      _p(ewt)))


def initial_step(mech, y0, t0, t_out, rtol, atol, T=1.0, kscale=None, F=None):
    """The integrator's initial step size for one cell; returns (h0, right-hand
    sides used)."""
    m = OracleMech(mech)
    o, atol_arr = _opts(rtol, atol)
    y0 = _f64(y0)
    nfe = C.c_int32(0)
    h0 = lib().orc_initial_step_cell(m.ptr, C.byref(o), float(T), _p(_f64(kscale)), _p(_f64(F)),
                                     float(t0), float(t_out), _p(y0), C.byref(nfe))
    return float(h0), int(nfe.value)


def steps(mech, kf, kr, z, q, h, hist0, F=None):
    """Fixed-order variable-coefficient BDF steps of prescribed sizes h[n] from
    the Nordsieck array z ([q+1][S], units of h[0]) with prior step sizes
    hist0 (hist0[k] = size of the (k+1)-th earlier step).  Correctors are
    solved to round-off.  Returns (y_n [n][S], e_n [n][S], Cerr_n [n], final z)."""
    m = OracleMech(mech)
    S = m.S
    kf, kr, F = _f64(kf), _f64(kr), _f64(F)
    h = _f64(np.atleast_1d(h))
    hist = np.zeros(QMAX + 1)
    hv = np.atleast_1d(np.asarray(hist0, dtype=np.float64))
    hist[: min(hv.size, QMAX + 1)] = hv[: QMAX + 1]
    zz = np.zeros((q + 1, S))
    zz[:] = np.asarray(z, dtype=np.float64)[: q + 1]
    n = h.size
    yo, eo, co = np.zeros((n, S)), np.zeros((n, S)), np.zeros(n)
    rc = lib().orc_steps(m.ptr, _p(kf), _p(kr), _p(F), int(q), n, _p(h), _p(hist), _p(zz), _p(yo),
                         _p(eo), _p(co))
    if rc:
        raise RuntimeError(f"steps failed: {rc}")
    return yo, eo, co, zz


def set_threads(n):
    """OpenMP threads of the batch integrations (0: leave unchanged)."""
    lib().orc_set_threads(int(n))


def splitmix64(x):
    return int(lib().orc_splitmix64(int(x) & 0xFFFFFFFFFFFFFFFF))


def perturb_uniform(seed, step, cell, species):
    return float(lib().orc_perturb_uniform(int(seed), int(step), int(cell), int(species)))


def perturb(y, n_species_of_cell, weights_of_cell, seed, step, amp, cell_index=None):
    """Returns a perturbed copy of y ([N][ldy]); row c is the cell with index
    cell_index[c] (default c) in the perturbation's key."""
    y = np.array(y, dtype=np.float64, order="C", copy=True)
    N, ldy = y.shape
    ns = np.ascontiguousarray(n_species_of_cell, dtype=np.int32)
    ws = [np.ascontiguousarray(w, dtype=np.float64) for w in weights_of_cell]
    ptrs = (C.c_void_p * N)()
    for c in range(N):
        ptrs[c] = ws[c].ctypes.data
    ci = None if cell_index is None else np.ascontiguousarray(cell_index, dtype=np.int64)
    lib().orc_perturb_cells(N, _p(ci), _p(ns), ldy, _p(y), C.cast(ptrs, C.c_void_p), int(seed),
                            int(step), float(amp))
    return y


def outer_loop(mechs, y0, cell_index, cell_mech, n_outer, dt, seed, amp, rtol, atol, T=None,
               integrate_seconds=None, **kw):
    """The operator-splitting outer loop on the cells ``cell_index`` of a
    batch (rows of y0, mechanisms cell_mech, temperatures T): for outer step
    k, perturb (keyed by the cells' own indices), then integrate over
    [k dt, (k+1) dt].  Returns (y, stats of the last step).  If
    ``integrate_seconds`` is a list, the wall time of each integration is
    appended to it (the perturbation is not timed)."""
    import time

    y = np.array(y0, dtype=np.float64, copy=True)
    S_of = [int(mechs[m]["n_species"]) for m in cell_mech]
    W_of = [mechs[m]["w"] for m in cell_mech]
    st = None
    for k in range(n_outer):
        y = perturb(y, S_of, W_of, seed, k, amp, cell_index=cell_index)
        t = time.perf_counter()
        y, st = integrate(mechs, y, k * dt, (k + 1) * dt, rtol, atol, T=T, cell_mech=cell_mech,
                          **kw)
        if integrate_seconds is not None:
            integrate_seconds.append(time.perf_counter() - t)
    return y, st


def typical_atol(y, eta, n_species, cell_mech=None):
    """Typical-value absolute tolerances (Sec. 4.1.3, Eq. (9)).

    For each mechanism m and species i < n_species[m], the typical value is
    half the sum of the smallest and largest y[c][i] over the cells c of
    mechanism m, and atol[m][i] = eta * typical.  Where the typical value is
    not positive (a species absent, or driven below zero, everywhere) the
    paper's default for unmanaged values, a typical value of 1, is used.
    Entries of a mechanism without cells, and beyond n_species[m], are left
    at eta and at 0 (typical).  Returns (typical [n_mech][ldy],
    atol [n_mech][ldy]); the arithmetic is 0.5 * (min + max), then * eta.
    """
    y = np.asarray(y, dtype=np.float64)
    N, ldy = y.shape
    n_species = [int(s) for s in np.atleast_1d(n_species)]
    n_mech = len(n_species)
    cm = np.zeros(N, dtype=np.int64) if cell_mech is None else np.asarray(cell_mech)
    typ = np.zeros((n_mech, ldy))
    atol = np.full((n_mech, ldy), float(eta))
    for m in range(n_mech):
        rows = y[cm == m]
        if rows.shape[0] == 0:
            continue
        for i in range(n_species[m]):
            lo, hi = np.min(rows[:, i]), np.max(rows[:, i])
            t = 0.5 * (lo + hi)
            typ[m, i] = t
            atol[m, i] = (t if t > 0.0 else 1.0) * float(eta)
    return typ, atol
