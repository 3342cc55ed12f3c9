"""ctypes front end of the plain-C FP64 oracle (``rb_oracle.c``).

TEST INFRASTRUCTURE ONLY (see the package docstring). Every function here marshals numpy
arrays into the C routines; the arithmetic lives in ``rb_oracle.c``.
"""

from __future__ import annotations

import ctypes as ct
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "rb_oracle.c")
LIB = os.path.join(HERE, "librb_oracle.so")

STATUS = {0: "converged", 1: "max_iter", 2: "singular", 3: "nonfinite", 4: "bad_n"}

_dp = ct.POINTER(ct.c_double)
_ip = ct.POINTER(ct.c_int)


class _Set(ct.Structure):
    _fields_ = [("Nm", ct.c_int), ("Q", ct.c_int), ("Qc", ct.c_int), ("Qf", ct.c_int),
                ("Npm", ct.c_int), ("Qb", ct.c_int),
                ("A", _dp), ("C", _dp), ("F", _dp), ("H", _dp),
                ("Bp", _dp), ("Asv", _dp), ("Csv", _dp), ("Fs", _dp)]


def build_oracle(force=False):
    """Compile rb_oracle.c with gcc (FP64, no FMA contraction, OpenMP)."""
    if not force and os.path.exists(LIB) and os.path.getmtime(LIB) >= os.path.getmtime(SRC):
        return LIB
    tmp = LIB + f".tmp{os.getpid()}"
    cmd = ["gcc", "-O2", "-std=c99", "-fopenmp", "-ffp-contract=off", "-fno-fast-math",
           "-shared", "-fPIC", "-o", tmp, SRC, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


_lib = None


def load_oracle():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
            build_oracle()
        lib = ct.CDLL(LIB)
        lib.orc_theta.argtypes = [ct.c_int] * 4 + [ct.c_double, ct.c_double] + [_dp] * 4
        lib.orc_theta.restype = ct.c_int
        lib.orc_gepp_solve.argtypes = [ct.c_int, _dp, _dp, _ip]
        lib.orc_gepp_solve.restype = ct.c_int
        lib.orc_newton.argtypes = [ct.POINTER(_Set), ct.c_int, _dp, _dp, _dp, _dp, ct.c_double,
                                   ct.c_int, _dp, _ip, _dp]
        lib.orc_newton.restype = ct.c_int
        lib.orc_picard.argtypes = [ct.POINTER(_Set), ct.c_int, _dp, _dp, _dp, ct.c_double,
                                   ct.c_int, _dp, _ip]
        lib.orc_picard.restype = ct.c_int
        lib.orc_pressure.argtypes = [ct.POINTER(_Set), ct.c_int, ct.c_int, _dp, _dp, _dp, _dp,
                                     _dp, _dp]
        lib.orc_pressure.restype = ct.c_int
        lib.orc_solve_batch.argtypes = [ct.POINTER(_Set), ct.c_int, _ip, _dp, _dp, _dp,
                                        ct.c_double, ct.c_int, _dp, _ip, _ip, ct.c_int, _dp,
                                        _ip, ct.c_int]
        lib.orc_solve_batch.restype = ct.c_int
        _lib = lib
    return _lib


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _ptr(a):
    return None if a is None else a.ctypes.data_as(_dp)


class OracleSet:
    """Holds FP64 copies of a tensor set and the C struct pointing at them."""

    def __init__(self, ts):
        self.N, self.Q, self.Qc, self.Qf = ts.N, ts.Q, ts.Qc, ts.Qf
        self.Np, self.Qb = ts.Np, ts.Qb
        self._keep = {k: _f64(getattr(ts, k)) for k in
                      ("A", "C", "F", "H", "Bp", "Asv", "Csv", "Fs")}
        if getattr(ts, "H", None) is None:
            self._keep["H"] = None
        k = self._keep
        self.s = _Set(ts.N, ts.Q, ts.Qc, ts.Qf, ts.Np, ts.Qb, _ptr(k["A"]), _ptr(k["C"]),
                      _ptr(k["F"]), _ptr(k["H"]), _ptr(k["Bp"]), _ptr(k["Asv"]),
                      _ptr(k["Csv"]), _ptr(k["Fs"]))


def theta(Q, Qc, Qf, Qb, alpha, Re):
    """theta^a, theta^c, theta^f, theta^b at one parameter (alpha in radians)."""
    lib = load_oracle()
    ta, tc, tf, tb = np.zeros(Q), np.zeros(Qc), np.zeros(Qf), np.zeros(Qb)
    rc = lib.orc_theta(Q, Qc, Qf, Qb, float(alpha), float(Re), _ptr(ta), _ptr(tc), _ptr(tf),
                       _ptr(tb))
    if rc != 0:
        raise ValueError("unsupported theta family sizes")
    return ta, tc, tf, tb


def gepp_solve(M, b, return_piv=False):
    """Solve M x = b with the oracle's partial-pivoting elimination."""
    lib = load_oracle()
    M = _f64(M).copy()
    x = _f64(b).copy()
    n = x.shape[0]
    piv = np.zeros(n, dtype=np.int32)
    st = lib.orc_gepp_solve(n, _ptr(M), _ptr(x), piv.ctypes.data_as(_ip))
    return (x, st, piv) if return_piv else (x, st)


def newton(oset, n, ta, tc, f, tol=1e-12, maxit=10, u0=None):
    """One Newton solve; returns (u, status, iters, update-norm history)."""
    lib = load_oracle()
    u = np.zeros(n)
    it = ct.c_int(0)
    hist = np.zeros(max(maxit, 1))
    st = lib.orc_newton(ct.byref(oset.s), n, _ptr(_f64(ta)), _ptr(_f64(tc)), _ptr(_f64(f)),
                        _ptr(None if u0 is None else _f64(u0)), tol, maxit, _ptr(u),
                        ct.byref(it), _ptr(hist))
    return u, st, it.value, hist[: it.value]


def picard(oset, n, ta, tc, f, tol=1e-15, maxit=500):
    lib = load_oracle()
    u = np.zeros(n)
    it = ct.c_int(0)
    st = lib.orc_picard(ct.byref(oset.s), n, _ptr(_f64(ta)), _ptr(_f64(tc)), _ptr(_f64(f)),
                        tol, maxit, _ptr(u), ct.byref(it))
    return u, st, it.value


def pressure(oset, n, npr, ta, tc, tf, tb, u):
    lib = load_oracle()
    p = np.zeros(npr)
    st = lib.orc_pressure(ct.byref(oset.s), n, npr, _ptr(_f64(ta)), _ptr(_f64(tc)),
                          _ptr(_f64(tf)), _ptr(_f64(tb)), _ptr(_f64(u)), _ptr(p))
    return p, st


def solve_batch(oset, mu, Nreq=None, fover=None, u0=None, tol=1e-12, maxit=10,
                pressure_np=0, nthreads=0):
    """Batch of solves (OpenMP). Returns dict with u [B,Nm], iters, status, p, pstatus."""
    lib = load_oracle()
    mu = _f64(mu)
    B = mu.shape[0]
    Nm = oset.N
    u = np.zeros((B, Nm))
    iters = np.zeros(B, dtype=np.int32)
    status = np.zeros(B, dtype=np.int32)
    p = np.zeros((B, oset.Np)) if pressure_np else None
    pst = np.zeros(B, dtype=np.int32)
    Nr = None if Nreq is None else np.ascontiguousarray(Nreq, dtype=np.int32)
    fo = None if fover is None else _f64(fover)
    uu = None if u0 is None else _f64(u0)
    used = lib.orc_solve_batch(
        ct.byref(oset.s), B, None if Nr is None else Nr.ctypes.data_as(_ip), _ptr(mu),
        _ptr(fo), _ptr(uu), tol, maxit, _ptr(u), iters.ctypes.data_as(_ip),
        status.ctypes.data_as(_ip), int(pressure_np), _ptr(p), pst.ctypes.data_as(_ip),
        int(nthreads))
    return dict(u=u, iters=iters, status=status, p=p, pstatus=pst, threads=used)
