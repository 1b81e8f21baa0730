"""Plain CPU FP64 oracle for the MG-MLQMC per-sample path.

TEST INFRASTRUCTURE ONLY.  Only the tests, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` may import this package; the product path
(the GPU library and its Python binding) never does, and shares no code with
it.  The C part (``oracle.c``) holds the sampler, KL field, discretisation,
direct solve and full multigrid; ``estimators.py`` holds the (quasi-)Monte
Carlo estimators.  ctypes marshalling only lives here.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

from . import build as _build
from .estimators import (  # noqa: F401  (re-exported)
    mlmc_estimate,
    upsilon,
    shift_statistics,
)

_HERE = os.path.dirname(os.path.abspath(__file__))
_lib = None
_variant = "default"

_dp = np.ctypeslib.ndpointer(dtype=np.float64, flags="C_CONTIGUOUS")
_ip = np.ctypeslib.ndpointer(dtype=np.int32, flags="C_CONTIGUOUS")
_u32p = np.ctypeslib.ndpointer(dtype=np.uint32, flags="C_CONTIGUOUS")
_u64p = np.ctypeslib.ndpointer(dtype=np.uint64, flags="C_CONTIGUOUS")


def select_build(variant: str) -> None:
    """Choose the oracle build before its first use: "default" (-O2, the
    tests) or "fast" (-O3 -march=native, the timed CPU baseline); the source
    and arithmetic are the same."""
    global _variant
    if variant not in _build.OPT:
        raise ValueError(variant)
    if _lib is not None and variant != _variant:
        raise RuntimeError("the oracle library is already loaded")
    if variant == "fast" and _lib is None:
        # -march=native: compile for the host that runs it, not the one that built the tree
        _build.build(force=True, variant="fast")
    _variant = variant


def lib():
    """Load (building first if stale) the oracle shared library."""
    global _lib
    if _lib is not None:
        return _lib
    path = _build.build(force=False, variant=_variant)
    L = C.CDLL(path)
    L.oracle_bitrev32.restype = C.c_uint32
    L.oracle_bitrev32.argtypes = [C.c_uint32]
    L.oracle_lattice_x.restype = None
    L.oracle_lattice_x.argtypes = [_u32p, C.c_int, _u64p, C.c_uint64, _u64p]
    L.oracle_unit.restype = C.c_double
    L.oracle_unit.argtypes = [C.c_uint64]
    L.oracle_norminv.restype = C.c_double
    L.oracle_norminv.argtypes = [C.c_double]
    L.oracle_points.restype = None
    L.oracle_points.argtypes = [_u32p, C.c_int, _u64p, C.c_int64, C.c_int64, _u64p, _dp]
    L.oracle_kl_root.restype = C.c_double
    L.oracle_kl_root.argtypes = [C.c_double, C.c_int]
    L.oracle_kl_theta.restype = C.c_double
    L.oracle_kl_theta.argtypes = [C.c_double, C.c_double]
    L.oracle_kl_psi.restype = C.c_double
    L.oracle_kl_psi.argtypes = [C.c_double, C.c_double, C.c_double]
    L.oracle_kl_modes.restype = C.c_int
    L.oracle_kl_modes.argtypes = [C.c_double, C.c_int, _ip, _ip, _dp]
    L.oracle_problem_new.restype = C.c_void_p
    L.oracle_problem_new.argtypes = [C.c_int, C.c_int, C.c_int, C.c_double, C.c_double,
                                     C.c_int, C.c_int, C.c_int, C.c_double, C.c_int]
    L.oracle_problem_free.restype = None
    L.oracle_problem_free.argtypes = [C.c_void_p]
    L.oracle_finest_mg_level.restype = C.c_int
    L.oracle_finest_mg_level.argtypes = [C.c_void_p, C.c_int]
    L.oracle_field_size.restype = C.c_int64
    L.oracle_field_size.argtypes = [C.c_void_p, C.c_int]
    L.oracle_field.restype = None
    L.oracle_field.argtypes = [C.c_void_p, _dp, C.c_int, _dp]
    L.oracle_apply.restype = None
    L.oracle_apply.argtypes = [C.c_int, _dp, _dp, _dp]
    L.oracle_direct_solve.restype = C.c_int
    L.oracle_direct_solve.argtypes = [C.c_int, _dp, _dp, _dp]
    L.oracle_qoi.restype = None
    L.oracle_qoi.argtypes = [C.c_int, _dp, C.POINTER(C.c_double), C.POINTER(C.c_double)]
    L.oracle_fmg.restype = C.c_int
    L.oracle_fmg.argtypes = [C.c_void_p, C.c_int, _dp, _dp, _ip, _dp, C.c_void_p,
                             C.c_void_p, C.c_void_p, C.c_int, C.POINTER(C.c_int)]
    L.oracle_sample_from_field.restype = C.c_int
    L.oracle_sample_from_field.argtypes = [C.c_void_p, C.c_int, _dp, C.c_int, _dp, _ip, _dp]
    L.oracle_sample.restype = C.c_int
    L.oracle_sample.argtypes = [C.c_void_p, C.c_int, _dp, C.c_int, _dp]
    L.oracle_batch.restype = C.c_int
    L.oracle_batch.argtypes = [C.c_void_p, C.c_int, C.c_int, _dp, C.c_int, _dp, C.c_int]
    L.oracle_restrict.restype = None
    L.oracle_restrict.argtypes = [C.c_int, _dp, _dp]
    L.oracle_prolong.restype = None
    L.oracle_prolong.argtypes = [C.c_int, _dp, _dp, C.c_int]
    L.oracle_rb_sweep.restype = None
    L.oracle_rb_sweep.argtypes = [C.c_int, _dp, _dp, _dp, C.c_int]
    L.oracle_vcycle.restype = C.c_int
    L.oracle_vcycle.argtypes = [C.c_void_p, C.c_int, _dp, _dp, _dp]
    _lib = L
    return L


# ---- Section 3.2: lattice sequence, shift, inverse normal -------------------
def bitrev32(v: int) -> int:
    return int(lib().oracle_bitrev32(int(v)))


def lattice_x(z: np.ndarray, delta: np.ndarray, n: int) -> np.ndarray:
    z = np.ascontiguousarray(z, dtype=np.uint32)
    delta = np.ascontiguousarray(delta, dtype=np.uint64)
    x = np.empty(len(z), dtype=np.uint64)
    lib().oracle_lattice_x(z, len(z), delta, int(n), x)
    return x


def unit(x: int) -> float:
    return float(lib().oracle_unit(int(x)))


def norminv(u: float) -> float:
    return float(lib().oracle_norminv(float(u)))


def points(z: np.ndarray, delta: np.ndarray, n_begin: int, n_end: int):
    """x [B][s] (uint64 fixed point) and y = Phi^-1(u(x)) [B][s]."""
    z = np.ascontiguousarray(z, dtype=np.uint32)
    delta = np.ascontiguousarray(delta, dtype=np.uint64)
    s = len(z)
    B = int(n_end) - int(n_begin)
    x = np.empty((B, s), dtype=np.uint64)
    y = np.empty((B, s), dtype=np.float64)
    lib().oracle_points(z, s, delta, int(n_begin), int(n_end), x, y)
    return x, y


# ---- Section 5: KL eigenpairs -----------------------------------------------
def kl_root(lam: float, k: int) -> float:
    return float(lib().oracle_kl_root(float(lam), int(k)))


def kl_theta(lam: float, w: float) -> float:
    return float(lib().oracle_kl_theta(float(lam), float(w)))


def kl_psi(lam: float, w: float, x: float) -> float:
    return float(lib().oracle_kl_psi(float(lam), float(w), float(x)))


def kl_modes(lam: float, s: int):
    """Ordered 2-D mode table: (i, j) 1-based and theta_i * theta_j."""
    mi = np.empty(s, dtype=np.int32)
    mj = np.empty(s, dtype=np.int32)
    th = np.empty(s, dtype=np.float64)
    if lib().oracle_kl_modes(float(lam), int(s), mi, mj, th) != 0:
        raise MemoryError("oracle_kl_modes")
    return mi, mj, th


# ---- Section 6: discretisation ---------------------------------------------
def apply(n: int, a: np.ndarray, u: np.ndarray) -> np.ndarray:
    a = np.ascontiguousarray(a, dtype=np.float64).reshape(-1)
    u = np.ascontiguousarray(u, dtype=np.float64).reshape(-1)
    out = np.empty(n * n)
    lib().oracle_apply(n, a, u, out)
    return out


def direct_solve(n: int, a: np.ndarray, f: np.ndarray) -> np.ndarray:
    a = np.ascontiguousarray(a, dtype=np.float64).reshape(-1)
    f = np.ascontiguousarray(f, dtype=np.float64).reshape(-1)
    u = np.empty(n * n)
    if lib().oracle_direct_solve(n, a, f, u) != 0:
        raise ArithmeticError("matrix not positive definite")
    return u


def qoi(n: int, u: np.ndarray):
    u = np.ascontiguousarray(u, dtype=np.float64).reshape(-1)
    qm, qc = C.c_double(), C.c_double()
    lib().oracle_qoi(n, u, C.byref(qm), C.byref(qc))
    return qm.value, qc.value


# ---- Section 4: pieces of the V-cycle --------------------------------------
def restrict(nc: int, r: np.ndarray) -> np.ndarray:
    """Mean of the four children: fine (2nc)^2 -> coarse nc^2."""
    r = np.ascontiguousarray(r, dtype=np.float64).reshape(-1)
    assert r.size == 4 * nc * nc
    fc = np.empty(nc * nc)
    lib().oracle_restrict(int(nc), r, fc)
    return fc


def prolong(nc: int, e: np.ndarray, out: np.ndarray | None = None) -> np.ndarray:
    """Bilinear prolongation of e (nc^2) to (2nc)^2; added to `out` if given."""
    e = np.ascontiguousarray(e, dtype=np.float64).reshape(-1)
    assert e.size == nc * nc
    add = out is not None
    o = np.ascontiguousarray(out, dtype=np.float64).reshape(-1).copy() if add else np.empty(4 * nc * nc)
    lib().oracle_prolong(int(nc), e, o, int(add))
    return o


def rb_sweep(n: int, a: np.ndarray, f: np.ndarray, u: np.ndarray, colour: int) -> np.ndarray:
    """One Gauss-Seidel half-sweep over the cells of `colour` (0 red); returns the new u."""
    a = np.ascontiguousarray(a, dtype=np.float64).reshape(-1)
    f = np.ascontiguousarray(f, dtype=np.float64).reshape(-1)
    u = np.ascontiguousarray(u, dtype=np.float64).reshape(-1).copy()
    lib().oracle_rb_sweep(int(n), a, f, u, int(colour))
    return u


class Problem:
    """One configured problem: n0, levels, KL (s, corr_len, sigma2) and the
    FMG cycle (mu0, mu1, mu2; rtol > 0 switches to refinement to rtol)."""

    def __init__(self, n0, num_levels, s, corr_len, sigma2, mu0=2, mu1=2, mu2=2,
                 rtol=0.0, max_iters=0):
        self.n0, self.num_levels, self.s = int(n0), int(num_levels), int(s)
        self.corr_len, self.sigma2 = float(corr_len), float(sigma2)
        self.mu0, self.mu1, self.mu2 = int(mu0), int(mu1), int(mu2)
        self.rtol, self.max_iters = float(rtol), int(max_iters)
        h = lib().oracle_problem_new(self.n0, self.num_levels, self.s, self.corr_len,
                                     self.sigma2, self.mu0, self.mu1, self.mu2,
                                     self.rtol, self.max_iters)
        if not h:
            raise ValueError("invalid oracle problem")
        self._h = C.c_void_p(h)
        self.g0 = int(np.log2(self.n0)) - 1

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and _lib is not None:
            _lib.oracle_problem_free(h)
            self._h = None

    def finest_mg_level(self, k: int) -> int:
        return int(lib().oracle_finest_mg_level(self._h, int(k)))

    def field_size(self, k: int) -> int:
        return int(lib().oracle_field_size(self._h, int(k)))

    def level_slices(self, k: int):
        """(g, n, slice) of every multigrid level 0..G in a level-major field."""
        out, off = [], 0
        for g in range(self.finest_mg_level(k) + 1):
            n = 2 << g
            out.append((g, n, slice(off, off + n * n)))
            off += n * n
        return out

    def vcycle(self, g: int, a_all: np.ndarray, u: np.ndarray, f: np.ndarray) -> np.ndarray:
        """One V(mu1, mu2) cycle on multigrid level g; a_all holds levels 0..g."""
        a_all = np.ascontiguousarray(a_all, dtype=np.float64).reshape(-1)
        n = 2 << g
        assert a_all.size == sum((2 << l) ** 2 for l in range(g + 1))
        u = np.ascontiguousarray(u, dtype=np.float64).reshape(-1).copy()
        f = np.ascontiguousarray(f, dtype=np.float64).reshape(-1)
        assert u.size == n * n and f.size == n * n
        if lib().oracle_vcycle(self._h, int(g), a_all, u, f) != 0:
            raise MemoryError("oracle_vcycle")
        return u

    def field(self, y: np.ndarray, k: int) -> np.ndarray:
        y = np.ascontiguousarray(y, dtype=np.float64).reshape(-1)
        assert y.size == self.s
        z = np.empty(self.field_size(k))
        lib().oracle_field(self._h, y, int(k), z)
        return z

    def fmg(self, G: int, a_all: np.ndarray, trace_cap: int = 0):
        a_all = np.ascontiguousarray(a_all, dtype=np.float64)
        q = np.empty(2 * (G + 1))
        it = np.empty(G + 1, dtype=np.int32)
        rr = np.empty(G + 1)
        nG = 2 << G
        u = np.empty(nG * nG)
        tr = np.zeros(max(trace_cap, 1), dtype=np.int32)
        mk = np.zeros(max(trace_cap, 1), dtype=np.int32)
        tl = C.c_int(0)
        st = lib().oracle_fmg(self._h, int(G), a_all, q, it, rr, u.ctypes.data,
                              tr.ctypes.data if trace_cap else None,
                              mk.ctypes.data if trace_cap else None,
                              int(trace_cap), C.byref(tl))
        res = dict(status=st, qoi=q.reshape(G + 1, 2), iters=it, relres=rr, u=u)
        if trace_cap:
            n = min(tl.value, trace_cap)
            res["trace"] = tr[:n].tolist()
            res["marks"] = mk[:n].tolist()
        return res

    def sample_from_field(self, k: int, z: np.ndarray, method: int = 0):
        z = np.ascontiguousarray(z, dtype=np.float64)
        q = np.empty(2 * (k + 1))
        it = np.empty(k + 1, dtype=np.int32)
        rr = np.empty(k + 1)
        st = lib().oracle_sample_from_field(self._h, int(k), z, int(method), q, it, rr)
        return dict(status=st, qoi=q.reshape(k + 1, 2), iters=it, relres=rr)

    def sample(self, k: int, y: np.ndarray, method: int = 0) -> np.ndarray:
        y = np.ascontiguousarray(y, dtype=np.float64).reshape(-1)
        q = np.empty(2 * (k + 1))
        lib().oracle_sample(self._h, int(k), y, int(method), q)
        return q.reshape(k + 1, 2)

    def batch(self, k: int, y: np.ndarray, method: int = 0, nthreads: int = 0):
        """QoI [B][k+1][2] (mean, centre) for B samples y [B][s]."""
        y = np.ascontiguousarray(y, dtype=np.float64)
        B = y.shape[0]
        q = np.empty((B, k + 1, 2))
        bad = lib().oracle_batch(self._h, int(k), int(B), y, int(method), q, int(nthreads))
        return q, int(bad)
