"""Python binding of libmlmc.so, the MI355X (gfx950) library for the per-sample
hot path of the multigrid multilevel (quasi-)Monte Carlo method.

Argument marshalling only: every step of the path runs in the library's HIP
kernels (or, for ``mlmc_estimate``, its host code).  PyTorch supplies device
memory and the current HIP stream.  There is no fallback: if the library is
missing, importing the entry points raises.

The names follow the C ABI in ``include/mlmc.h``: ``mlmc_create``,
``mlmc_destroy``, ``mlmc_points_gen``, ``mlmc_field``, ``mlmc_fmg_solve``,
``mlmc_estimate``, ``mlmc_kl_modes``, ``mlmc_fmg_trace`` ...; ``Context`` wraps
them for torch tensors.
"""
from __future__ import annotations

import ctypes as C
import os
import threading
import time

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmlmc.so")

MLMC_OK, MLMC_E_INVAL, MLMC_E_NOMEM, MLMC_E_HIP, MLMC_E_NOCONV, MLMC_E_STATE = 0, -1, -2, -3, -4, -5
MLMC_FP64, MLMC_MIXED = 0, 1
MLMC_QOI_MEAN, MLMC_QOI_CENTER = 1, 2
MLMC_POINTS_LATTICE, MLMC_POINTS_EXPLICIT = 0, 1
MLMC_PASS_TILE32, MLMC_PASS_TILE16, MLMC_PASS_STREAM = 0, 1, 2
MLMC_FIELD_SEPARABLE_EXP, MLMC_FIELD_MATERN = 0, 1
MLMC_BATCH_CLASSES = 10


class mlmc_config(C.Structure):
    _fields_ = [("n0", C.c_int32), ("num_levels", C.c_int32), ("s", C.c_int32),
                ("corr_len", C.c_double), ("sigma2", C.c_double),
                ("mu0", C.c_int32), ("mu1", C.c_int32), ("mu2", C.c_int32),
                ("rtol", C.c_double), ("max_iters", C.c_int32), ("precision", C.c_int32),
                ("qoi_mask", C.c_uint32), ("num_shifts", C.c_int32),
                ("genvec", C.c_void_p), ("shifts", C.c_void_p), ("max_batch", C.c_int64),
                ("field_kind", C.c_int32), ("nu", C.c_double), ("nystrom_q", C.c_int32)]


class mlmc_points(C.Structure):
    _fields_ = [("kind", C.c_int32), ("level", C.c_int32), ("shift_begin", C.c_int32),
                ("shift_end", C.c_int32), ("n_begin", C.c_int64), ("n_end", C.c_int64),
                ("y_dev", C.c_void_p)]


class mlmc_solve_info(C.Structure):
    _fields_ = [("samples", C.c_int64), ("max_iters_used", C.c_int32),
                ("max_rel_residual", C.c_double), ("not_converged", C.c_int64)]


class mlmc_profile_result(C.Structure):
    _fields_ = [("launches", C.c_int64), ("total_ms", C.c_double), ("bytes", C.c_double),
                ("flops", C.c_double)]


class mlmc_tune_entry(C.Structure):
    _fields_ = [("n", C.c_int32), ("batch_class", C.c_int32), ("pre", C.c_int32),
                ("post", C.c_int32), ("pre_ms", C.c_double), ("post_ms", C.c_double)]


MLMC_KERNEL = dict(points=0, field=1, smooth=2, restrict=3, prolong=4, coarse=5, qoi=6, sums=7,
                   pre=8, post=9, lds=10, refine=11)


class mlmc_est_input(C.Structure):
    _fields_ = [("num_levels", C.c_int32), ("num_shifts", C.c_int32), ("nq", C.c_int32),
                ("reuse", C.c_int32), ("n_per_level", C.c_void_p), ("sums", C.c_void_p)]


class mlmc_est_output(C.Structure):
    _fields_ = [("upsilon", C.c_void_p), ("upsilon_bar", C.c_void_p), ("var_level", C.c_void_p),
                ("q_shift", C.c_void_p), ("q_bar", C.c_void_p), ("var_q", C.c_void_p)]


class mlmc_request(C.Structure):
    _fields_ = [("level", C.c_int32), ("shift_begin", C.c_int32), ("shift_end", C.c_int32),
                ("n_begin", C.c_int64), ("n_end", C.c_int64), ("tag", C.c_uint64),
                ("qoi_out", C.c_void_p), ("sums_out", C.c_void_p)]


class mlmc_result(C.Structure):
    _fields_ = [("tag", C.c_uint64), ("status", C.c_int32), ("level", C.c_int32),
                ("samples", C.c_int64), ("batch_samples", C.c_int64),
                ("queued_ms", C.c_double), ("latency_ms", C.c_double),
                ("not_converged", C.c_int64), ("max_rel_residual", C.c_double)]


class mlmc_server_stats(C.Structure):
    _fields_ = [("requests", C.c_int64), ("samples", C.c_int64), ("batches", C.c_int64),
                ("p50_ms", C.c_double), ("p99_ms", C.c_double), ("max_ms", C.c_double),
                ("busy_s", C.c_double)]


EXPORTS = [
    "mlmc_create", "mlmc_destroy", "mlmc_field_size", "mlmc_num_qoi", "mlmc_points_gen",
    "mlmc_field", "mlmc_fmg_solve", "mlmc_estimate", "mlmc_kl_modes", "mlmc_fmg_trace",
    "mlmc_status_str", "mlmc_last_error", "mlmc_profile_begin", "mlmc_profile_end",
    "mlmc_server_create", "mlmc_server_destroy", "mlmc_server_submit", "mlmc_server_poll",
    "mlmc_server_stats_get", "mlmc_server_capacity", "mlmc_autotune", "mlmc_tuning_get",
    "mlmc_tuning_set", "mlmc_field_static",
]

_lib = None


class MlmcError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{msg} (status {status})")
        self.status = status


def lib():
    """Load libmlmc.so; raises if it has not been built (no fallback path)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with __graft_entry__.build()")
    L = C.CDLL(LIB_PATH)
    vp, i32, i64 = C.c_void_p, C.c_int32, C.c_int64
    sig = {
        "mlmc_create": (i32, [C.POINTER(mlmc_config), C.c_int, C.POINTER(vp)]),
        "mlmc_destroy": (i32, [vp]),
        "mlmc_field_size": (i64, [vp, i32]),
        "mlmc_num_qoi": (i32, [vp]),
        "mlmc_points_gen": (i32, [vp, C.POINTER(mlmc_points), vp, vp, vp]),
        "mlmc_field": (i32, [vp, C.POINTER(mlmc_points), vp, vp]),
        "mlmc_field_static": (i32, [vp, C.POINTER(mlmc_points), vp, vp]),
        "mlmc_fmg_solve": (i32, [vp, C.POINTER(mlmc_points), vp, vp, vp,
                                 C.POINTER(mlmc_solve_info), vp]),
        "mlmc_estimate": (i32, [C.POINTER(mlmc_est_input), C.POINTER(mlmc_est_output)]),
        "mlmc_kl_modes": (i32, [vp, vp, vp, vp]),
        "mlmc_fmg_trace": (i32, [vp, i32, vp, vp, i64, C.POINTER(i64)]),
        "mlmc_profile_begin": (i32, [vp, i32]),
        "mlmc_profile_end": (i32, [vp, C.POINTER(mlmc_profile_result)]),
        "mlmc_server_create": (i32, [C.POINTER(mlmc_config), C.c_int, i32, i64, C.POINTER(vp)]),
        "mlmc_server_destroy": (i32, [vp]),
        "mlmc_server_submit": (i32, [vp, C.POINTER(mlmc_request)]),
        "mlmc_server_poll": (i32, [vp, C.POINTER(mlmc_result), i32, i32, C.POINTER(i32)]),
        "mlmc_server_stats_get": (i32, [vp, C.POINTER(mlmc_server_stats)]),
        "mlmc_server_capacity": (i64, [vp, i32]),
        "mlmc_autotune": (i32, [vp, i32, vp]),
        "mlmc_tuning_get": (i32, [vp, C.POINTER(mlmc_tune_entry), i32, C.POINTER(i32)]),
        "mlmc_tuning_set": (i32, [vp, C.POINTER(mlmc_tune_entry), i32]),
        "mlmc_status_str": (C.c_char_p, [i32]),
        "mlmc_last_error": (C.c_char_p, [vp]),
    }
    for name, (res, args) in sig.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    _lib = L
    return L


def _check(st, ctx=None):
    if st != MLMC_OK:
        L = lib()
        msg = (L.mlmc_last_error(ctx) or b"").decode() or L.mlmc_status_str(st).decode()
        raise MlmcError(st, msg)
    return st


def mlmc_estimate(n_per_level, sums, num_shifts, nq, reuse):
    """Host estimator (no GPU).  sums: float64 [L+1][R][nq][L+1][2]."""
    n_per_level = np.ascontiguousarray(n_per_level, dtype=np.int64)
    sums = np.ascontiguousarray(sums, dtype=np.float64)
    L1 = len(n_per_level)
    assert sums.shape == (L1, num_shifts, nq, L1, 2), sums.shape
    out = dict(upsilon=np.zeros((nq, L1, num_shifts)), upsilon_bar=np.zeros((nq, L1)),
               var_level=np.zeros((nq, L1)), q_shift=np.zeros((nq, num_shifts)),
               q_bar=np.zeros(nq), var_q=np.zeros(nq))
    inp = mlmc_est_input(L1, int(num_shifts), int(nq), int(bool(reuse)),
                         n_per_level.ctypes.data, sums.ctypes.data)
    o = mlmc_est_output(*(out[k].ctypes.data for k in
                          ("upsilon", "upsilon_bar", "var_level", "q_shift", "q_bar", "var_q")))
    _check(lib().mlmc_estimate(C.byref(inp), C.byref(o)))
    return out


def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


def _stream():
    import torch
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _config(n0, num_levels, s, corr_len, sigma2, mu0, mu1, mu2, rtol, max_iters, precision,
            qoi_mask, genvec, shifts, max_batch, field_kind=MLMC_FIELD_SEPARABLE_EXP, nu=0.5,
            nystrom_q=0):
    """mlmc_config plus the host arrays it points to (kept alive by the caller)."""
    genvec = None if genvec is None else np.ascontiguousarray(genvec, dtype=np.uint32)
    shifts = None if shifts is None else np.ascontiguousarray(shifts, dtype=np.uint64)
    R = 0 if shifts is None else int(shifts.shape[1])
    cfg = mlmc_config(int(n0), int(num_levels), int(s), float(corr_len), float(sigma2),
                      int(mu0), int(mu1), int(mu2), float(rtol), int(max_iters),
                      int(precision), int(qoi_mask), R,
                      None if genvec is None else genvec.ctypes.data,
                      None if shifts is None else shifts.ctypes.data,
                      int(max_batch), int(field_kind), float(nu), int(nystrom_q))
    return cfg, genvec, shifts


class Context:
    """An mlmc_ctx bound to one device; tensors must live on that device."""

    def __init__(self, n0, num_levels, s, corr_len, sigma2, mu0=2, mu1=2, mu2=2, rtol=0.0,
                 max_iters=0, precision=MLMC_FP64, qoi_mask=MLMC_QOI_MEAN, genvec=None,
                 shifts=None, max_batch=1024, device=0, field_kind=MLMC_FIELD_SEPARABLE_EXP,
                 nu=0.5, nystrom_q=0):
        cfg, self._genvec, self._shifts = _config(n0, num_levels, s, corr_len, sigma2, mu0, mu1,
                                                  mu2, rtol, max_iters, precision, qoi_mask,
                                                  genvec, shifts, max_batch, field_kind, nu,
                                                  nystrom_q)
        R = cfg.num_shifts
        h = C.c_void_p()
        _check(lib().mlmc_create(C.byref(cfg), int(device), C.byref(h)))
        self._h = h
        self.cfg = cfg
        self.device = device
        self.nq = int(lib().mlmc_num_qoi(h))
        self.num_shifts = R

    def close(self):
        if getattr(self, "_h", None):
            lib().mlmc_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    # ---- helpers -----------------------------------------------------------
    def _stream(self):
        return None if self.device < 0 else _stream()

    @staticmethod
    def lattice(level, n_begin, n_end, shift_begin=0, shift_end=1):
        return mlmc_points(MLMC_POINTS_LATTICE, int(level), int(shift_begin), int(shift_end),
                           int(n_begin), int(n_end), None)

    @staticmethod
    def explicit(level, y, replica=0):
        pts = mlmc_points(MLMC_POINTS_EXPLICIT, int(level), int(replica), int(replica) + 1, 0,
                          int(y.shape[0]), y.data_ptr())
        pts._y = y          # keep the device buffer alive as long as the points
        return pts

    @staticmethod
    def count(pts):
        return (pts.n_end - pts.n_begin) * (pts.shift_end - pts.shift_begin)

    def field_size(self, level):
        return int(lib().mlmc_field_size(self._h, int(level)))

    # ---- entry points ------------------------------------------------------
    def points_gen(self, pts, x=None, y=None):
        _check(lib().mlmc_points_gen(self._h, C.byref(pts), _ptr(x), _ptr(y), self._stream()), self._h)

    def field(self, pts, z):
        _check(lib().mlmc_field(self._h, C.byref(pts), _ptr(z), self._stream()), self._h)

    def field_static(self, pts, z):
        """mlmc_field_static: the field with no allocation (static scratch)."""
        _check(lib().mlmc_field_static(self._h, C.byref(pts), _ptr(z), self._stream()), self._h)

    def fmg_solve(self, pts, z=None, qoi=None, sums=None, want_info=False):
        info = mlmc_solve_info()
        st = lib().mlmc_fmg_solve(self._h, C.byref(pts), _ptr(z), _ptr(qoi), _ptr(sums),
                                  C.byref(info) if want_info else None, self._stream())
        if st != MLMC_E_NOCONV:
            _check(st, self._h)
        if want_info:
            return dict(status=st, samples=info.samples, max_iters_used=info.max_iters_used,
                        max_rel_residual=info.max_rel_residual, not_converged=info.not_converged)
        return None

    def profile_begin(self, kind):
        _check(lib().mlmc_profile_begin(self._h, int(MLMC_KERNEL[kind])), self._h)

    def profile_end(self):
        r = mlmc_profile_result()
        _check(lib().mlmc_profile_end(self._h, C.byref(r)), self._h)
        return dict(launches=r.launches, total_ms=r.total_ms, bytes=r.bytes, flops=r.flops)

    def autotune(self, level=None):
        """Measure the pass kinds of every tile grid up to `level` (default:
        the finest) and batch class on this context's stream; install the
        fastest.  Returns the table (see tuning())."""
        lev = self.cfg.num_levels - 1 if level is None else int(level)
        _check(lib().mlmc_autotune(self._h, lev, self._stream()), self._h)
        return self.tuning()

    def tuning(self):
        """The pass-kind table: dicts n, batch_class, pre, post, pre_ms, post_ms."""
        cnt = C.c_int32(0)
        _check(lib().mlmc_tuning_get(self._h, None, 0, C.byref(cnt)), self._h)
        arr = (mlmc_tune_entry * max(cnt.value, 1))()
        _check(lib().mlmc_tuning_get(self._h, arr, cnt.value, C.byref(cnt)), self._h)
        return [dict(n=e.n, batch_class=e.batch_class, pre=e.pre, post=e.post, pre_ms=e.pre_ms,
                     post_ms=e.post_ms) for e in arr[:cnt.value]]

    def set_tuning(self, entries):
        """Install pass kinds: an iterable of dicts with n, batch_class, pre, post."""
        entries = list(entries)
        arr = (mlmc_tune_entry * max(len(entries), 1))()
        for k, e in enumerate(entries):
            arr[k] = mlmc_tune_entry(int(e["n"]), int(e["batch_class"]), int(e["pre"]),
                                     int(e["post"]), 0.0, 0.0)
        _check(lib().mlmc_tuning_set(self._h, arr, len(entries)), self._h)

    def kl_modes(self):
        s = self.cfg.s
        i = np.empty(s, dtype=np.int32)
        j = np.empty(s, dtype=np.int32)
        t = np.empty(s, dtype=np.float64)
        _check(lib().mlmc_kl_modes(self._h, i.ctypes.data, j.ctypes.data, t.ctypes.data), self._h)
        return i, j, t

    def fmg_trace(self, level, cap=100000):
        lv = np.zeros(cap, dtype=np.int32)
        mk = np.zeros(cap, dtype=np.int32)
        n = C.c_int64(0)
        _check(lib().mlmc_fmg_trace(self._h, int(level), lv.ctypes.data, mk.ctypes.data, cap,
                                    C.byref(n)), self._h)
        n = min(n.value, cap)
        return lv[:n].tolist(), mk[:n].tolist()


class Server:
    """mlmc_server: slots of one configuration serving solve requests from a
    FIFO with same-level batching.  QoIs come back in host arrays
    [B][level+1][nq] owned by this object until the result is polled."""

    def __init__(self, n0, num_levels, s, corr_len, sigma2, genvec, shifts, mu0=2, mu1=2, mu2=2,
                 rtol=0.0, max_iters=0, precision=MLMC_FP64, qoi_mask=MLMC_QOI_MEAN,
                 num_slots=2, slot_samples=1024, device=0, field_kind=MLMC_FIELD_SEPARABLE_EXP,
                 nu=0.5, nystrom_q=0):
        cfg, self._genvec, self._shifts = _config(n0, num_levels, s, corr_len, sigma2, mu0, mu1,
                                                  mu2, rtol, max_iters, precision, qoi_mask,
                                                  genvec, shifts, slot_samples, field_kind, nu,
                                                  nystrom_q)
        h = C.c_void_p()
        _check(lib().mlmc_server_create(C.byref(cfg), int(device), int(num_slots),
                                        int(slot_samples), C.byref(h)))
        self._h = h
        self.cfg = cfg
        self.nq = bin(int(qoi_mask) & 3).count("1")
        self.slot_samples = int(slot_samples)
        self._pending = {}
        self._done = {}
        self._lat = []
        self._next_tag = 0
        self._lock = threading.RLock()

    def submit(self, level, n_begin, n_end, shift_begin=0, shift_end=1, tag=None, sums=False):
        """Queue lattice points [n_begin, n_end) of shifts [shift_begin,
        shift_end) on finest level `level`; returns the request's tag.  With
        sums=True the result also carries the per-shift level-difference sums
        [shift_end - shift_begin][nq][level+1][2] formed by the library."""
        with self._lock:
            if tag is None:
                tag = self._next_tag
            tag = int(tag)
            if tag in self._pending or tag in self._done:
                raise ValueError(f"tag {tag} is still pending")
            self._next_tag = max(self._next_tag, tag + 1)
            B = max(0, (int(n_end) - int(n_begin)) * (int(shift_end) - int(shift_begin)))
            out = np.zeros((B, int(level) + 1, self.nq), dtype=np.float64)
            so = (np.zeros((max(0, int(shift_end) - int(shift_begin)), self.nq, int(level) + 1, 2))
                  if sums else None)
            req = mlmc_request(int(level), int(shift_begin), int(shift_end), int(n_begin),
                               int(n_end), tag, out.ctypes.data if B else None,
                               so.ctypes.data if so is not None and so.size else None)
            _check(lib().mlmc_server_submit(self._h, C.byref(req)))
            self._pending[tag] = (out, so)
            return tag

    def poll(self, max_results=256, wait_ms=0):
        """Completed requests, oldest first: dicts with the result fields,
        'qoi' (the request's array) and 'sums' (None unless requested)."""
        buf = (mlmc_result * max(1, int(max_results)))()
        n = C.c_int32(0)
        _check(lib().mlmc_server_poll(self._h, buf, int(max_results), int(wait_ms), C.byref(n)))
        res = []
        with self._lock:
            for r in buf[: n.value]:
                qoi, sums = self._pending.pop(int(r.tag))
                res.append(dict(tag=int(r.tag), status=int(r.status), level=int(r.level),
                                samples=int(r.samples), batch_samples=int(r.batch_samples),
                                queued_ms=r.queued_ms, latency_ms=r.latency_ms,
                                not_converged=int(r.not_converged),
                                max_rel_residual=float(r.max_rel_residual),
                                qoi=qoi, sums=sums))
                self._lat.append(r.latency_ms)
        return res

    def take_latencies(self):
        """Latencies (ms) of the requests polled since the last call."""
        with self._lock:
            lat, self._lat = self._lat, []
        return lat

    def collect(self, tags, timeout_s=600.0):
        """Wait for the results of `tags` (safe from several threads: results
        polled for other callers are kept for them); returns them in order."""
        t0 = time.monotonic()
        while True:
            with self._lock:
                for r in self.poll(max_results=1024, wait_ms=0):
                    self._done[r["tag"]] = r
                if all(t in self._done for t in tags):
                    return [self._done.pop(t) for t in tags]
            if time.monotonic() - t0 > timeout_s:
                raise TimeoutError(f"{len(tags)} requests not completed in {timeout_s} s")
            time.sleep(2e-4)

    def pending(self):
        with self._lock:
            return len(self._pending)

    def capacity(self, level):
        """Samples of `level` one batch holds (requests may not exceed it)."""
        return int(lib().mlmc_server_capacity(self._h, int(level)))

    def stats(self):
        st = mlmc_server_stats()
        _check(lib().mlmc_server_stats_get(self._h, C.byref(st)))
        return {k: getattr(st, k) for k, _ in mlmc_server_stats._fields_}

    def close(self):
        """Finishes queued requests, then frees the slots."""
        if getattr(self, "_h", None):
            lib().mlmc_server_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()
