"""CPU FP64 oracle of the interpolated pseudodifferential Helmholtz preconditioner.

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the benchmark's CPU
baseline leg may import this package; the HIP product path never does.  The
arithmetic lives in plain C (``helm_oracle.c``), written from the paper, and is
called through ctypes on numpy arrays.  Nothing here is shared with the HIP
library.

Parity pins of every function are in ``tests/test_oracle_*.py``.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "helm_oracle.c")
_LIB = os.path.join(_HERE, "libhelm_oracle.so")

OK, E_INVALID, E_SHAPE, E_MEDIA, E_LAYER, E_NOMEM, E_NOT_CONVERGED = 0, 1, 2, 3, 4, 7, 8


_LIB_OMP = os.path.join(_HERE, "libhelm_oracle_omp.so")


def build(force: bool = False, openmp: bool = False) -> str:
    """Compile the oracle with gcc, -O2: single-threaded (the library the tests use), or
    with OpenMP over its independent loops (transform lines, points, the reductions of
    the Gram-Schmidt dot products), used only to time the oracle on every host core."""
    lib_path = _LIB_OMP if openmp else _LIB
    if force or not os.path.exists(lib_path) or os.path.getmtime(lib_path) < os.path.getmtime(_SRC):
        tmp = lib_path + ".tmp%d" % os.getpid()
        extra = ["-fopenmp"] if openmp else []
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", *extra, "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, lib_path)
    return lib_path


class _Problem(C.Structure):
    _fields_ = [("dim", C.c_int), ("n", C.c_int * 3), ("len", C.c_double * 3),
                ("omega", C.c_double), ("c", C.c_void_p), ("a", C.c_void_p), ("zeta", C.c_void_p),
                ("c0", C.c_double), ("m_real", C.c_int), ("m_layer", C.c_int), ("symbol", C.c_int),
                ("a_floor", C.c_double), ("nodes_real", C.c_void_p), ("nodes_zeta", C.c_void_p),
                ("a_nodes", C.c_void_p), ("interp_order", C.c_int), ("m_damp", C.c_int),
                ("layer_tensor", C.c_int)]


class _Setup(C.Structure):
    _fields_ = [("M", C.c_int), ("Mt", C.c_int), ("K", C.c_int), ("mo", C.c_int),
                ("cmin", C.c_double), ("cmax", C.c_double), ("zmax", C.c_double),
                ("cnode", C.c_double * 64), ("znode", C.c_double * 65), ("ahat", C.c_double * 64),
                ("gre", C.c_double * 64), ("gim", C.c_double * 64), ("order", C.c_int),
                ("Ma", C.c_int), ("anode", C.c_double * 64), ("amin", C.c_double), ("amax", C.c_double),
                ("tensor", C.c_int)]


class _Info(C.Structure):
    _fields_ = [("iters", C.c_int), ("cycles", C.c_int), ("rel_true_residual", C.c_double),
                ("status", C.c_int), ("rel_prec_residual", C.c_double)]


_lib = None
_lib_omp = None
_use_openmp = False


def use_openmp(on: bool) -> int:
    """Route the oracle's calls to the OpenMP build (on) or the single-threaded one;
    returns the threads the selected library uses."""
    global _use_openmp
    _use_openmp = bool(on)
    return int(lib().or_num_threads())


def lib():
    global _lib, _lib_omp
    if _use_openmp:
        if _lib_omp is None:
            _lib_omp = C.CDLL(build(openmp=True))
            assert _lib_omp.or_setup_sizeof() == C.sizeof(_Setup)
        return _lib_omp
    if _lib is None:
        _lib = C.CDLL(build())
        assert _lib.or_setup_sizeof() == C.sizeof(_Setup)
        assert _lib.or_problem_sizeof() == C.sizeof(_Problem)
    return _lib


class OracleError(RuntimeError):
    def __init__(self, code, what):
        super().__init__(f"{what}: oracle status {code}")
        self.code = code


def _ptr(a):
    return None if a is None else C.c_void_p(a.ctypes.data)


def _addr(a):
    return None if a is None else a.ctypes.data


class Problem:
    """A Helmholtz problem on a periodic grid plus the preconditioner options.

    c, a, zeta: real arrays of the grid shape (a, zeta optional).
    symbol: "continuous" (|xi|^2, Eqn. 021) or "discrete" (the stencil's own symbol).
    """

    def __init__(self, shape, omega, c, a=None, zeta=None, length=1.0, c0=1.0, m_real=8,
                 m_layer=3, symbol="continuous", a_floor=0.0, nodes_real=None,
                 nodes_zeta=None, a_nodes=None, interp_order=1, m_damp=0, layer_tensor=False):
        self.shape = tuple(int(s) for s in shape)
        self.dim = len(self.shape)
        self.c = np.ascontiguousarray(c, dtype=np.float64).reshape(self.shape)
        self.a = None if a is None else np.ascontiguousarray(a, dtype=np.float64).reshape(self.shape)
        self.zeta = None if zeta is None else np.ascontiguousarray(zeta, dtype=np.float64).reshape(self.shape)
        self.nodes_real = None if nodes_real is None else np.ascontiguousarray(nodes_real, dtype=np.float64)
        self.nodes_zeta = None if nodes_zeta is None else np.ascontiguousarray(nodes_zeta, dtype=np.float64)
        self.a_nodes = None if a_nodes is None else np.ascontiguousarray(a_nodes, dtype=np.float64)
        p = _Problem()
        p.dim = self.dim
        for d in range(self.dim):
            p.n[d] = self.shape[d]
            p.len[d] = float(length)
        p.omega = float(omega)
        p.c, p.a, p.zeta = _addr(self.c), _addr(self.a), _addr(self.zeta)
        p.c0 = float(c0)
        p.m_real = int(m_real if nodes_real is None else len(nodes_real))
        p.m_layer = int(m_layer if nodes_zeta is None else len(nodes_zeta))
        p.symbol = {"continuous": 0, "discrete": 1}[symbol]
        p.a_floor = float(a_floor)
        p.nodes_real, p.nodes_zeta, p.a_nodes = _addr(self.nodes_real), _addr(self.nodes_zeta), _addr(self.a_nodes)
        p.interp_order = int(interp_order)
        p.m_damp = int(m_damp)
        p.layer_tensor = int(bool(layer_tensor))
        self._p = p
        self.omega = float(omega)
        self.length = float(length)
        self.c0 = float(c0)

    @property
    def npts(self):
        return int(np.prod(self.shape))

    def setup(self):
        s = _Setup()
        rc = lib().or_setup(C.byref(self._p), C.byref(s))
        if rc:
            raise OracleError(rc, "setup")
        K = s.K
        return {"M": s.M, "Mt": s.Mt, "K": K, "mo": s.mo, "cmin": s.cmin, "cmax": s.cmax,
                "zmax": s.zmax, "cnode": np.array(s.cnode[:s.M]), "znode": np.array(s.znode[:s.Mt + 1]),
                "ahat": np.array(s.ahat[:K]), "gamma": np.array(s.gre[:K]) + 1j * np.array(s.gim[:K]),
                "Ma": s.Ma, "anode": np.array(s.anode[:s.Ma]), "tensor": s.tensor, "_raw": s}

    def weights(self, cval, zval):
        """All K node weights at a point with wave speed cval and layer value zval."""
        st = self.setup()
        w = (C.c_double * 128)()
        lib().or_point_weights(C.byref(st["_raw"]), C.c_double(self.c0), C.c_double(cval),
                               C.c_double(zval), w)
        return np.array(w[:st["K"]])

    def weights_ca(self, cval, aval):
        """The M x Ma node weights of the bivariate (c, a) scheme at a point."""
        st = self.setup()
        w = (C.c_double * 128)()
        lib().or_point_weights_ca(C.byref(st["_raw"]), C.c_double(cval), C.c_double(aval), w)
        return np.array(w[:st["K"]])

    def _fields(self, x):
        x = np.ascontiguousarray(x, dtype=np.complex128)
        if x.shape == self.shape:
            return x[None], True
        assert x.shape[1:] == self.shape, (x.shape, self.shape)
        return x, False

    def apply(self, v):
        """u = Q_M v (Eqn. 403)."""
        v, single = self._fields(v)
        u = np.empty_like(v)
        rc = lib().or_apply(C.byref(self._p), C.c_int(v.shape[0]), _ptr(v), _ptr(u))
        if rc:
            raise OracleError(rc, "apply")
        return u[0] if single else u

    def matvec(self, u):
        """y = P_N u (second-order centred differences, periodic)."""
        u, single = self._fields(u)
        y = np.empty_like(u)
        rc = lib().or_matvec(C.byref(self._p), C.c_int(u.shape[0]), _ptr(u), _ptr(y))
        if rc:
            raise OracleError(rc, "matvec")
        return y[0] if single else y

    def exact_psdo(self, v):
        """Brute-force exact operator Q of Eqn. Precond (small grids only)."""
        v = np.ascontiguousarray(v, dtype=np.complex128).reshape(self.shape)
        u = np.empty_like(v)
        rc = lib().or_exact_psdo(C.byref(self._p), _ptr(v), _ptr(u))
        if rc:
            raise OracleError(rc, "exact_psdo")
        return u

    def arnoldi(self, v0, m, side="right", reorth=False):
        v0 = np.ascontiguousarray(v0, dtype=np.complex128).reshape(self.shape)
        V = np.zeros((m + 1,) + self.shape, dtype=np.complex128)
        H = np.zeros((m + 1, m), dtype=np.complex128)
        steps = C.c_int(0)
        rc = lib().or_arnoldi(C.byref(self._p), C.c_int(_SIDE[side]), C.c_int(m), C.c_int(int(reorth)), _ptr(v0),
                              _ptr(V), _ptr(H), C.byref(steps))
        if rc:
            raise OracleError(rc, "arnoldi")
        return V, H, steps.value

    def gmres(self, f, x0=None, restart=30, max_cycles=200, rtol=1e-8, side="right", hist_len=1000):
        f = np.ascontiguousarray(f, dtype=np.complex128).reshape(self.shape)
        x = np.zeros_like(f) if x0 is None else np.array(x0, dtype=np.complex128).reshape(self.shape)
        info = _Info()
        hist = np.zeros(hist_len)
        rc = lib().or_gmres(C.byref(self._p), C.c_int(_SIDE[side]), C.c_int(restart),
                            C.c_int(max_cycles), C.c_double(rtol), _ptr(f), _ptr(x), C.byref(info),
                            _ptr(hist), C.c_int(hist_len))
        if rc not in (OK, E_NOT_CONVERGED):
            raise OracleError(rc, "gmres")
        res = {"iters": info.iters, "cycles": info.cycles, "rel_true_residual": info.rel_true_residual,
               "rel_prec_residual": info.rel_prec_residual, "status": info.status,
               "history": hist[:max(1, info.cycles + 1)]}
        return x, res


_SIDE = {"right": 0, "left": 1, "none": 2}


def fft1d(x, sign=-1):
    x = np.array(x, dtype=np.complex128)
    rc = lib().or_fft1d(C.c_int(x.size), _ptr(x), C.c_int(sign))
    if rc:
        raise OracleError(rc, "fft1d")
    return x


def dft1d_naive(x, sign=-1):
    x = np.ascontiguousarray(x, dtype=np.complex128)
    y = np.empty_like(x)
    lib().or_dft1d_naive(C.c_int(x.size), _ptr(x), _ptr(y), C.c_int(sign))
    return y


def fftnd(x, inverse=False):
    x = np.array(x, dtype=np.complex128)
    n = (C.c_int * 3)(*(list(x.shape) + [1] * (3 - x.ndim)))
    rc = lib().or_fftnd(C.c_int(x.ndim), n, _ptr(x), C.c_int(1 if inverse else 0))
    if rc:
        raise OracleError(rc, "fftnd")
    return x


def from_workload(w, symbol="continuous", **over):
    """Oracle problem for a synthetic workload."""
    kw = dict(length=w.length, c0=w.c0, m_real=w.m_real, m_layer=w.m_layer, symbol=symbol,
              a_floor=w.a_floor)
    kw.update(over)
    return Problem(w.shape, w.omega, w.c, w.a, w.zeta, **kw)
