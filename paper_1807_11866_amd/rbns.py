"""ctypes binding of librbns.so (the C ABI in include/rbns.h).

Argument marshalling only: every step of the online solve runs in the HIP library. PyTorch
provides device memory (tensors) and the current HIP stream; nothing here computes on the
host. If the shared library is missing the import of this module's functions fails loudly:
there is no CPU fallback.
"""

from __future__ import annotations

import ctypes as ct
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "librbns.so")

RB_OK, RB_E_INVAL, RB_E_NOMEM, RB_E_DEVICE, RB_E_STATE, RB_E_UNSUPPORTED = 0, -1, -2, -3, -4, -5
RB_ST_CONVERGED, RB_ST_MAXIT, RB_ST_SINGULAR, RB_ST_NONFINITE, RB_ST_BADN = 0, 1, 2, 3, 4
RB_PREC_F64, RB_PREC_F32, RB_PREC_BF16, RB_PREC_BF16X3 = 0, 1, 2, 3

EXPORTED = ("rb_create", "rb_destroy", "rb_last_error", "rb_hbm_used", "rb_load_tensors",
            "rb_theta", "rb_solve_batch", "rb_solve_batch_noalloc", "rb_solve_uneven", "rb_autotune", "rb_tuned_config",
            "rb_recover_pressure", "rb_recover_pressure_uneven", "rb_reconstruct_pressure",
            "rb_assemble_convection", "rb_server_start", "rb_server_submit", "rb_server_poll",
            "rb_server_stats", "rb_server_stop", "rb_timing_enable", "rb_timing_read")
RB_ST_FAILED = 5
RB_ST_REFINED = 6
RB_MAX_N, RB_MAX_NP = 152, 64

_dp = ct.POINTER(ct.c_double)
_vp = ct.c_void_p


class RbError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"rbns error {code}: {msg}")
        self.code = code


class TensorsDesc(ct.Structure):
    _fields_ = [("N", ct.c_int), ("Q", ct.c_int), ("Qc", ct.c_int), ("Qf", ct.c_int),
                ("A", _dp), ("C", _dp), ("F", _dp), ("H", _dp),
                ("Np", ct.c_int), ("Qb", ct.c_int),
                ("Bp", _dp), ("Asv", _dp), ("Csv", _dp), ("Fs", _dp)]


class SolveOpts(ct.Structure):
    _fields_ = [("tol", ct.c_double), ("max_iter", ct.c_int), ("precision", ct.c_int),
                ("refine_steps", ct.c_int)]


class ServerOpts(ct.Structure):
    _fields_ = [("precision", ct.c_int), ("refine_steps", ct.c_int), ("max_iter", ct.c_int),
                ("tol", ct.c_double), ("max_batch", ct.c_int), ("lanes", ct.c_int),
                ("hbm_budget_bytes", ct.c_size_t), ("pressure", ct.c_int)]


class Request(ct.Structure):
    _fields_ = [("alpha", ct.c_double), ("re", ct.c_double), ("N", ct.c_int),
                ("tag", ct.c_longlong)]


class Result(ct.Structure):
    _fields_ = [("ticket", ct.c_longlong), ("tag", ct.c_longlong), ("N", ct.c_int),
                ("status", ct.c_int), ("iters", ct.c_int), ("pstatus", ct.c_int),
                ("latency_ms", ct.c_double), ("queue_ms", ct.c_double),
                ("u", ct.c_double * RB_MAX_N),
                ("p", ct.c_double * RB_MAX_NP)]


class ServerStats(ct.Structure):
    _fields_ = [("submitted", ct.c_longlong), ("completed", ct.c_longlong),
                ("batches", ct.c_longlong), ("p50_ms", ct.c_double), ("p99_ms", ct.c_double),
                ("max_ms", ct.c_double), ("p50_queue_ms", ct.c_double),
                ("p99_queue_ms", ct.c_double), ("mean_batch", ct.c_double),
                ("first_submit_s", ct.c_double), ("last_done_s", ct.c_double),
                ("hbm_inflight_peak", ct.c_size_t), ("error", ct.c_char * 256)]


_lib = None


def load(path=None):
    """Load librbns.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    path = path or LIB_PATH
    if not os.path.exists(path):
        raise RuntimeError(f"{path} not found: build it with `python -m paper_1807_11866_amd.build`"
                           " (there is no CPU fallback)")
    lib = ct.CDLL(path)
    lib.rb_create.argtypes = [ct.c_int, ct.c_size_t, ct.POINTER(_vp)]
    lib.rb_destroy.argtypes = [_vp]
    lib.rb_last_error.restype = ct.c_char_p
    lib.rb_hbm_used.argtypes = [_vp]
    lib.rb_hbm_used.restype = ct.c_size_t
    lib.rb_load_tensors.argtypes = [_vp, ct.POINTER(TensorsDesc), ct.POINTER(ct.c_int)]
    lib.rb_theta.argtypes = [_vp, ct.c_int, ct.c_int] + [_vp] * 5 + [_vp]
    lib.rb_solve_batch.argtypes = ([_vp, ct.c_int, ct.c_int, ct.c_int, ct.c_int] + [_vp] * 5 +
                                   [ct.POINTER(SolveOpts)] + [_vp] * 3 + [_vp])
    lib.rb_solve_batch_noalloc.argtypes = lib.rb_solve_batch.argtypes
    lib.rb_solve_uneven.argtypes = ([_vp, ct.c_int, ct.c_int, _vp, ct.c_int] + [_vp] * 5 +
                                    [ct.POINTER(SolveOpts)] + [_vp] * 3 + [_vp])
    lib.rb_autotune.argtypes = ([_vp, ct.c_int, ct.c_int, ct.c_int] + [_vp] * 3 +
                                [ct.POINTER(SolveOpts), _vp])
    lib.rb_tuned_config.argtypes = [_vp, ct.c_int, ct.c_int, ct.c_int, ct.c_int,
                                    ct.POINTER(ct.c_int), ct.POINTER(ct.c_int)]
    lib.rb_recover_pressure.argtypes = ([_vp] + [ct.c_int] * 6 + [_vp] * 7 + [_vp])
    lib.rb_recover_pressure_uneven.argtypes = ([_vp, ct.c_int, ct.c_int, _vp] + [ct.c_int] * 3 +
                                               [_vp] * 7 + [_vp])
    lib.rb_reconstruct_pressure.argtypes = ([_vp, ct.c_int, ct.c_int, ct.c_int, _vp, ct.c_int,
                                             _vp, ct.c_int, _vp, ct.c_int, _vp])
    lib.rb_assemble_convection.argtypes = ([_vp] + [ct.c_int] * 4 + [_vp] * 4 +
                                           [ct.c_double, _vp, _vp])
    lib.rb_server_start.argtypes = [_vp, ct.c_int, ct.POINTER(ServerOpts), ct.POINTER(_vp)]
    lib.rb_server_submit.argtypes = [_vp, ct.POINTER(Request), ct.c_int,
                                     ct.POINTER(ct.c_longlong)]
    lib.rb_server_poll.argtypes = [_vp, ct.POINTER(Result), ct.c_int, ct.POINTER(ct.c_int)]
    lib.rb_server_stats.argtypes = [_vp, ct.POINTER(ServerStats)]
    lib.rb_server_stop.argtypes = [_vp]
    lib.rb_timing_enable.argtypes = [_vp, ct.c_int]
    lib.rb_timing_read.argtypes = [_vp, ct.c_char_p, ct.POINTER(ct.c_double),
                                   ct.POINTER(ct.c_int)]
    for fn in EXPORTED:
        if fn not in ("rb_last_error", "rb_hbm_used"):
            getattr(lib, fn).restype = ct.c_int
    _lib = lib
    return lib


def _check(rc):
    if rc != RB_OK:
        raise RbError(rc, load().rb_last_error().decode())
    return rc


def _ptr(t):
    """Device (or host) address of a torch tensor / numpy array, or None."""
    if t is None:
        return None
    if hasattr(t, "data_ptr"):
        return ct.c_void_p(t.data_ptr())
    return ct.c_void_p(t.ctypes.data)


def _stream(stream):
    if stream is None:
        import torch
        return ct.c_void_p(torch.cuda.current_stream().cuda_stream)
    if hasattr(stream, "cuda_stream"):
        return ct.c_void_p(stream.cuda_stream)
    return ct.c_void_p(stream)


# ---------------------------------------------------------------- thin C mirrors ---------

def rb_create(device=0, hbm_budget_bytes=0):
    ctx = _vp()
    _check(load().rb_create(int(device), int(hbm_budget_bytes), ct.byref(ctx)))
    return ctx


def rb_destroy(ctx):
    _check(load().rb_destroy(ctx))


def rb_hbm_used(ctx):
    return load().rb_hbm_used(ctx)


def rb_load_tensors(ctx, ts):
    """Copy a tensor set (numpy FP64 arrays, see rbinputs.TensorSet) to the device."""
    import numpy as np

    keep = {}

    def p(name):
        a = getattr(ts, name, None)
        if a is None:
            return None
        a = np.ascontiguousarray(a, dtype=np.float64)
        keep[name] = a
        return a.ctypes.data_as(_dp)

    npr = int(getattr(ts, "Np", 0) or 0)
    d = TensorsDesc(int(ts.N), int(ts.Q), int(ts.Qc), int(ts.Qf), p("A"), p("C"), p("F"),
                    p("H"), npr, int(getattr(ts, "Qb", 1) or 1),
                    p("Bp") if npr else None, p("Asv") if npr else None,
                    p("Csv") if npr else None, p("Fs") if npr else None)
    sid = ct.c_int(-1)
    _check(load().rb_load_tensors(ctx, ct.byref(d), ct.byref(sid)))
    return sid.value


def rb_theta(ctx, set_id, B, mu, theta_a, theta_c, theta_f, theta_b=None, stream=None):
    _check(load().rb_theta(ctx, set_id, int(B), _ptr(mu), _ptr(theta_a), _ptr(theta_c),
                           _ptr(theta_f), _ptr(theta_b), _stream(stream)))


def make_opts(tol=1e-12, max_iter=10, precision=RB_PREC_F64, refine_steps=1):
    return SolveOpts(float(tol), int(max_iter), int(precision), int(refine_steps))


def rb_solve_batch(ctx, set_id, B, N, ldu, theta_a, theta_c, theta_f, f_override, u0, opts,
                   u, iters, status, stream=None):
    _check(load().rb_solve_batch(ctx, set_id, int(B), int(N), int(ldu), _ptr(theta_a),
                                 _ptr(theta_c), _ptr(theta_f), _ptr(f_override), _ptr(u0),
                                 ct.byref(opts) if opts is not None else None, _ptr(u),
                                 _ptr(iters), _ptr(status), _stream(stream)))


def rb_solve_batch_noalloc(ctx, set_id, B, N, ldu, theta_a, theta_c, theta_f, f_override, u0,
                           opts, u, iters, status, stream=None):
    _check(load().rb_solve_batch_noalloc(ctx, set_id, int(B), int(N), int(ldu), _ptr(theta_a),
                                         _ptr(theta_c), _ptr(theta_f), _ptr(f_override),
                                         _ptr(u0), ct.byref(opts) if opts is not None else None,
                                         _ptr(u), _ptr(iters), _ptr(status), _stream(stream)))


def rb_solve_uneven(ctx, set_id, B, N, ldu, theta_a, theta_c, theta_f, f_override, u0, opts,
                    u, iters, status, stream=None):
    _check(load().rb_solve_uneven(ctx, set_id, int(B), _ptr(N), int(ldu), _ptr(theta_a),
                                  _ptr(theta_c), _ptr(theta_f), _ptr(f_override), _ptr(u0),
                                  ct.byref(opts) if opts is not None else None, _ptr(u),
                                  _ptr(iters), _ptr(status), _stream(stream)))


def rb_autotune(ctx, set_id, B, N, theta_a, theta_c, theta_f, opts, stream=None):
    _check(load().rb_autotune(ctx, set_id, int(B), int(N), _ptr(theta_a), _ptr(theta_c),
                              _ptr(theta_f), ct.byref(opts) if opts is not None else None,
                              _stream(stream)))


def rb_tuned_config(ctx, set_id, N, precision, B):
    """(row splits per tile, LU variant 0 = readlane / 1 = LDS) used for such a batch."""
    ns, lv = ct.c_int(0), ct.c_int(0)
    _check(load().rb_tuned_config(ctx, set_id, int(N), int(precision), int(B), ct.byref(ns),
                                  ct.byref(lv)))
    return ns.value, lv.value


def rb_recover_pressure(ctx, set_id, B, N, Np, ldu, ldp, theta_a, theta_c, theta_f, theta_b,
                        u, p, status, stream=None):
    _check(load().rb_recover_pressure(ctx, set_id, int(B), int(N), int(Np), int(ldu),
                                      int(ldp), _ptr(theta_a), _ptr(theta_c), _ptr(theta_f),
                                      _ptr(theta_b), _ptr(u), _ptr(p), _ptr(status),
                                      _stream(stream)))


def rb_recover_pressure_uneven(ctx, set_id, B, N, Np, ldu, ldp, theta_a, theta_c, theta_f,
                               theta_b, u, p, status, stream=None):
    _check(load().rb_recover_pressure_uneven(ctx, set_id, int(B), _ptr(N), int(Np), int(ldu),
                                             int(ldp), _ptr(theta_a), _ptr(theta_c),
                                             _ptr(theta_f), _ptr(theta_b), _ptr(u), _ptr(p),
                                             _ptr(status), _stream(stream)))


def rb_reconstruct_pressure(ctx, B, N, Np, Pc, ldpc, u, ldu, p, ldp, stream=None):
    _check(load().rb_reconstruct_pressure(ctx, int(B), int(N), int(Np), _ptr(Pc), int(ldpc),
                                          _ptr(u), int(ldu), _ptr(p), int(ldp),
                                          _stream(stream)))


def rb_assemble_convection(ctx, N, R, X, Qc, phiT, dphiT, testT, M, w, out, stream=None):
    """M: host FP64 array [Qc][2][2]; the other arrays device tensors (layouts in rbns.h)."""
    import numpy as np
    Mh = np.ascontiguousarray(M, dtype=np.float64)
    _check(load().rb_assemble_convection(ctx, int(N), int(R), int(X), int(Qc), _ptr(phiT),
                                         _ptr(dphiT), _ptr(testT), _ptr(Mh), float(w),
                                         _ptr(out), _stream(stream)))


def rb_timing_enable(ctx, enable=True):
    _check(load().rb_timing_enable(ctx, int(bool(enable))))


def rb_timing_read(ctx, family):
    """(total milliseconds, launches) of the timed launches of one kernel family."""
    ms = ct.c_double(0.0)
    n = ct.c_int(0)
    _check(load().rb_timing_read(ctx, family.encode(), ct.byref(ms), ct.byref(n)))
    return ms.value, n.value


# ---------------------------------------------------------------- convenience ------------

class Solver:
    """One context + one loaded tensor set, with torch-allocated per-call buffers."""

    def __init__(self, ts, device=0, hbm_budget_bytes=0):
        import torch

        self.torch = torch
        self.dev = torch.device("cuda", device)
        self.ctx = rb_create(device, hbm_budget_bytes)
        self.set = rb_load_tensors(self.ctx, ts)
        self.N, self.Q, self.Qc, self.Qf = ts.N, ts.Q, ts.Qc, ts.Qf
        self.Np, self.Qb = int(getattr(ts, "Np", 0) or 0), int(getattr(ts, "Qb", 1) or 1)

    def close(self):
        if self.ctx:
            rb_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def theta(self, mu, stream=None):
        t = self.torch
        B = mu.shape[0]
        f64 = dict(dtype=t.float64, device=self.dev)
        th = dict(ta=t.empty(B, self.Q, **f64), tc=t.empty(B, self.Qc, **f64),
                  tf=t.empty(B, self.Qf, **f64),
                  tb=t.empty(B, self.Qb, **f64) if self.Np else None)
        rb_theta(self.ctx, self.set, B, mu, th["ta"], th["tc"], th["tf"], th["tb"], stream)
        return th

    def solve(self, th, N=None, f_override=None, u0=None, tol=1e-12, max_iter=10,
              precision=RB_PREC_F64, refine_steps=1, out=None, stream=None):
        t = self.torch
        N = self.N if N is None else N
        B = th["ta"].shape[0]
        if out is None:
            out = dict(u=t.empty(B, self.N, dtype=t.float64, device=self.dev),
                       iters=t.empty(B, dtype=t.int32, device=self.dev),
                       status=t.empty(B, dtype=t.int32, device=self.dev))
        opts = make_opts(tol, max_iter, precision, refine_steps)
        rb_solve_batch(self.ctx, self.set, B, N, self.N, th["ta"], th["tc"], th["tf"],
                       f_override, u0, opts, out["u"], out["iters"], out["status"], stream)
        return out

    def solve_uneven(self, th, Nreq, f_override=None, u0=None, tol=1e-12, max_iter=10,
                     precision=RB_PREC_F64, refine_steps=1, out=None, stream=None):
        t = self.torch
        B = th["ta"].shape[0]
        if out is None:
            out = dict(u=t.empty(B, self.N, dtype=t.float64, device=self.dev),
                       iters=t.empty(B, dtype=t.int32, device=self.dev),
                       status=t.empty(B, dtype=t.int32, device=self.dev))
        opts = make_opts(tol, max_iter, precision, refine_steps)
        rb_solve_uneven(self.ctx, self.set, B, Nreq, self.N, th["ta"], th["tc"], th["tf"],
                        f_override, u0, opts, out["u"], out["iters"], out["status"], stream)
        return out

    def pressure_uneven(self, th, u, Nreq, Np=None, out=None, stream=None):
        t = self.torch
        Np = self.Np if Np is None else Np
        B = u.shape[0]
        if out is None:
            out = dict(p=t.empty(B, self.Np, dtype=t.float64, device=self.dev),
                       pstatus=t.empty(B, dtype=t.int32, device=self.dev))
        rb_recover_pressure_uneven(self.ctx, self.set, B, Nreq, Np, u.shape[1], self.Np,
                                   th["ta"], th["tc"], th["tf"], th["tb"], u, out["p"],
                                   out["pstatus"], stream)
        return out

    def autotune(self, th, N=None, tol=1e-12, max_iter=10, precision=RB_PREC_F64,
                 refine_steps=1, stream=None):
        N = self.N if N is None else N
        rb_autotune(self.ctx, self.set, th["ta"].shape[0], N, th["ta"], th["tc"], th["tf"],
                    make_opts(tol, max_iter, precision, refine_steps), stream)
        return rb_tuned_config(self.ctx, self.set, N, precision, th["ta"].shape[0])

    def reconstruct(self, Pc, u, N=None, out=None, stream=None):
        """Pressure from a combined basis: p = Pc[:, :N] u (Pc a device [Np][>= N] array)."""
        t = self.torch
        N = self.N if N is None else N
        Np = Pc.shape[0]
        B = u.shape[0]
        if out is None:
            out = t.empty(B, Np, dtype=t.float64, device=self.dev)
        rb_reconstruct_pressure(self.ctx, B, N, Np, Pc, Pc.shape[1], u, u.shape[1], out,
                                out.shape[1], stream)
        return out

    def pressure(self, th, u, N=None, Np=None, out=None, stream=None):
        t = self.torch
        N = self.N if N is None else N
        Np = self.Np if Np is None else Np
        B = u.shape[0]
        if out is None:
            out = dict(p=t.empty(B, self.Np, dtype=t.float64, device=self.dev),
                       pstatus=t.empty(B, dtype=t.int32, device=self.dev))
        rb_recover_pressure(self.ctx, self.set, B, N, Np, u.shape[1], self.Np, th["ta"],
                            th["tc"], th["tf"], th["tb"], u, out["p"], out["pstatus"], stream)
        return out


class Server:
    """Continuous-batching server (rb_server_*) over a Solver's context and tensor set."""

    def __init__(self, solver, precision=RB_PREC_F64, refine_steps=1, max_iter=10, tol=1e-12,
                 max_batch=1024, lanes=3, hbm_budget_bytes=0, pressure=False):
        self.solver = solver
        o = ServerOpts(int(precision), int(refine_steps), int(max_iter), float(tol),
                       int(max_batch), int(lanes), int(hbm_budget_bytes), int(bool(pressure)))
        self.h = _vp()
        _check(load().rb_server_start(solver.ctx, solver.set, ct.byref(o), ct.byref(self.h)))
        self._buf = (Result * 4096)()

    _REQ = None

    @classmethod
    def _req_dtype(cls):
        import numpy as np
        if cls._REQ is None:
            cls._REQ = np.dtype({"names": ["alpha", "re", "N", "tag"],
                                 "formats": ["<f8", "<f8", "<i4", "<i8"],
                                 "offsets": [Request.alpha.offset, Request.re.offset,
                                             Request.N.offset, Request.tag.offset],
                                 "itemsize": ct.sizeof(Request)})
        return cls._REQ

    def submit(self, alpha, re, N, tags=None):
        """Queue requests (arrays of equal length, or scalars broadcast); returns their
        tickets (numpy int64)."""
        import numpy as np
        alpha = np.atleast_1d(np.asarray(alpha, dtype=np.float64))
        n = alpha.shape[0]
        reqs = np.zeros(n, dtype=self._req_dtype())
        reqs["alpha"] = alpha
        reqs["re"] = np.broadcast_to(np.asarray(re, dtype=np.float64), (n,))
        reqs["N"] = np.broadcast_to(np.asarray(N, dtype=np.int32), (n,))
        reqs["tag"] = np.arange(n) if tags is None else np.broadcast_to(np.asarray(tags), (n,))
        tk = np.empty(n, dtype=np.int64)
        _check(load().rb_server_submit(self.h, reqs.ctypes.data_as(ct.POINTER(Request)), n,
                                       tk.ctypes.data_as(ct.POINTER(ct.c_longlong))))
        return tk

    def poll_array(self):
        """Finished results as a numpy structured array with the fields of rb_result."""
        import numpy as np
        parts = []
        while True:
            n = ct.c_int(0)
            _check(load().rb_server_poll(self.h, self._buf, len(self._buf), ct.byref(n)))
            if n.value:
                parts.append(np.ctypeslib.as_array(self._buf)[:n.value].copy())
            if n.value < len(self._buf):
                break
        if not parts:
            return np.ctypeslib.as_array(self._buf)[:0].copy()
        return np.concatenate(parts)

    def poll(self):
        """Finished results as a list of dicts (ticket, tag, N, status, iters, pstatus,
        latency_ms, queue_ms, u (first N entries), p)."""
        out = []
        for r in self.poll_array():
            out.append(dict(ticket=int(r["ticket"]), tag=int(r["tag"]), N=int(r["N"]),
                            status=int(r["status"]), iters=int(r["iters"]),
                            pstatus=int(r["pstatus"]), latency_ms=float(r["latency_ms"]),
                            queue_ms=float(r["queue_ms"]),
                            u=r["u"][:int(r["N"])].copy(), p=r["p"].copy()))
        return out

    def stats(self):
        st = ServerStats()
        _check(load().rb_server_stats(self.h, ct.byref(st)))
        d = {k: getattr(st, k) for k, _ in ServerStats._fields_}
        d["error"] = st.error.decode()
        return d

    def stop(self):
        if self.h:
            _check(load().rb_server_stop(self.h))
            self.h = None
