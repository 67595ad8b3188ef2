"""Thin ctypes binding of libhelmpre.so (the C ABI declared in include/helmpre.h).

Only argument marshalling happens here: every step of the preconditioner, the
stencil and the solver runs in the HIP library.  PyTorch provides the device
memory (tensors on the GPU) and the stream.  If the library is not built, or no
GPU is present, the calls raise: there is no fallback.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libhelmpre.so")

HP_OK, HP_E_INVALID, HP_E_SHAPE, HP_E_MEDIA, HP_E_LAYER = 0, 1, 2, 3, 4
HP_E_NONFINITE, HP_E_DEVICE, HP_E_NOMEM, HP_E_NOT_CONVERGED = 5, 6, 7, 8
HP_FP64, HP_MIXED = 0, 1
SYMBOLS = {"continuous": 0, "discrete": 1}
PRECISIONS = {"fp64": HP_FP64, "mixed": HP_MIXED}

EXPORTED = ["hp_plan_create", "hp_plan_workspace_bytes", "hp_solve_workspace_bytes", "hp_plan_query",
            "hp_apply_precond", "hp_matvec", "hp_solve", "hp_profile_apply", "hp_plan_destroy",
            "hp_status_str", "hp_last_error", "hp_solver_create", "hp_solver_start", "hp_solver_advance",
            "hp_solver_wait", "hp_solver_destroy", "hp_arnoldi", "hp_ritz_values",
            "hp_arnoldi_vector", "hp_extreme_eigenvalue", "hp_plan_autotune", "hp_plan_time_pass",
            "hp_plan_pass_times", "hp_apply_precond_static", "hp_solver_advance_group"]


class HpGrid(C.Structure):
    _fields_ = [("dim", C.c_int), ("n", C.c_int * 3), ("len", C.c_double * 3)]


class HpLayer(C.Structure):
    _fields_ = [("zeta", C.c_void_p), ("c0", C.c_double)]


class HpPlanOpts(C.Structure):
    _fields_ = [("m_real", C.c_int), ("m_layer", C.c_int), ("nodes_real", C.c_void_p),
                ("nodes_zeta", C.c_void_p), ("a_nodes", C.c_void_p), ("a_floor", C.c_double),
                ("symbol", C.c_int), ("precision", C.c_int), ("max_nrhs", C.c_int), ("interp_order", C.c_int),
                ("m_damp", C.c_int), ("layer_tensor", C.c_int)]


SIDES = {"right": 0, "left": 1, "none": 2}   # HP_RIGHT, HP_LEFT, HP_NONE
# operators of the spectral diagnostics: the sides, plus (Q P_N)^{-1} and P_N^{-1}
ARNOLDI_OPS = dict(SIDES, left_inverse=3, none_inverse=4)


class HpSolveOpts(C.Structure):
    _fields_ = [("restart", C.c_int), ("max_cycles", C.c_int), ("rtol", C.c_double), ("side", C.c_int)]


class HpSolveInfo(C.Structure):
    _fields_ = [("iters", C.c_int), ("cycles", C.c_int), ("rel_true_residual", C.c_double),
                ("status", C.c_int), ("rel_prec_residual", C.c_double)]


class HpPlanInfo(C.Structure):
    _fields_ = [("dim", C.c_int), ("n", C.c_int * 3), ("K", C.c_int), ("M", C.c_int), ("Mt", C.c_int),
                ("mo", C.c_int), ("cmin", C.c_double), ("cmax", C.c_double), ("zeta_max", C.c_double),
                ("cnode", C.c_double * 64), ("znode", C.c_double * 65), ("ahat", C.c_double * 64),
                ("gamma_re", C.c_double * 64), ("gamma_im", C.c_double * 64),
                ("workspace_bytes", C.c_size_t), ("precision", C.c_int), ("interp_order", C.c_int),
                ("m_damp", C.c_int), ("anode", C.c_double * 64), ("tune", (C.c_int * 4) * 5),
                ("layer_tensor", C.c_int)]


_lib = None


def load_library(path: str = LIB_PATH):
    """Load libhelmpre.so (raises OSError if it is not built)."""
    global _lib
    if _lib is not None:
        return _lib
    # PyTorch ships its own HIP runtime; it must be the one in the process before this
    # library is mapped, so that both share one runtime (tensors, streams).
    import torch  # noqa: F401
    if not os.path.exists(path):
        raise OSError(f"{path} is not built; run __graft_entry__.build() or "
                      "python paper_2409_16172_amd/build.py")
    lib = C.CDLL(path)
    vp, i, d, sz = C.c_void_p, C.c_int, C.c_double, C.c_size_t
    lib.hp_plan_create.argtypes = [C.POINTER(vp), C.POINTER(HpGrid), d, vp, vp, C.POINTER(HpLayer),
                                   C.POINTER(HpPlanOpts), vp]
    lib.hp_plan_create.restype = i
    lib.hp_plan_workspace_bytes.argtypes = [C.POINTER(HpGrid), C.POINTER(HpPlanOpts), i]
    lib.hp_plan_workspace_bytes.restype = sz
    lib.hp_solve_workspace_bytes.argtypes = [C.POINTER(HpGrid), i, i]
    lib.hp_solve_workspace_bytes.restype = sz
    lib.hp_plan_query.argtypes = [vp, C.POINTER(HpPlanInfo)]
    lib.hp_plan_query.restype = i
    lib.hp_apply_precond.argtypes = [vp, vp, vp, i, vp]
    lib.hp_apply_precond.restype = i
    lib.hp_apply_precond_static.argtypes = [vp, vp, vp, i, vp]
    lib.hp_apply_precond_static.restype = i
    lib.hp_matvec.argtypes = [vp, vp, vp, i, vp]
    lib.hp_matvec.restype = i
    lib.hp_solve.argtypes = [vp, vp, vp, i, C.POINTER(HpSolveOpts), C.POINTER(HpSolveInfo), vp]
    lib.hp_solve.restype = i
    lib.hp_profile_apply.argtypes = [vp, vp, vp, i, i, C.POINTER(d), C.POINTER(d), vp]
    lib.hp_profile_apply.restype = i
    lib.hp_plan_time_pass.argtypes = [vp, i]
    lib.hp_plan_time_pass.restype = i
    lib.hp_plan_pass_times.argtypes = [vp, C.POINTER(d), i, C.POINTER(i)]
    lib.hp_plan_pass_times.restype = i
    lib.hp_arnoldi.argtypes = [vp, vp, i, i, vp, C.POINTER(i), vp]
    lib.hp_arnoldi.restype = i
    lib.hp_ritz_values.argtypes = [vp, i, i, i, vp, vp, C.POINTER(d)]
    lib.hp_ritz_values.restype = i
    lib.hp_plan_autotune.argtypes = [vp, C.POINTER(d), C.POINTER(d), vp]
    lib.hp_plan_autotune.restype = i
    lib.hp_arnoldi_vector.argtypes = [vp, vp, i, vp, vp]
    lib.hp_arnoldi_vector.restype = i
    lib.hp_extreme_eigenvalue.argtypes = [vp, vp, i, i, i, i, d, vp, C.POINTER(d), C.POINTER(i), vp]
    lib.hp_extreme_eigenvalue.restype = i
    lib.hp_solver_create.argtypes = [C.POINTER(vp), vp, i, C.POINTER(HpSolveOpts)]
    lib.hp_solver_create.restype = i
    lib.hp_solver_start.argtypes = [vp, vp, vp, vp]
    lib.hp_solver_start.restype = i
    lib.hp_solver_advance.argtypes = [vp, i, C.POINTER(i)]
    lib.hp_solver_advance.restype = i
    lib.hp_solver_advance_group.argtypes = [C.POINTER(vp), i, i, C.POINTER(i)]
    lib.hp_solver_advance_group.restype = i
    lib.hp_solver_wait.argtypes = [vp, C.POINTER(HpSolveInfo)]
    lib.hp_solver_wait.restype = i
    lib.hp_solver_destroy.argtypes = [vp]
    lib.hp_solver_destroy.restype = i
    lib.hp_plan_destroy.argtypes = [vp]
    lib.hp_plan_destroy.restype = i
    lib.hp_status_str.argtypes = [i]
    lib.hp_status_str.restype = C.c_char_p
    lib.hp_last_error.argtypes = []
    lib.hp_last_error.restype = C.c_char_p
    _lib = lib
    return lib


class HelmpreError(RuntimeError):
    def __init__(self, code: int, where: str):
        lib = load_library()
        msg = lib.hp_status_str(code).decode()
        detail = lib.hp_last_error().decode() if code in (HP_E_DEVICE, HP_E_NOMEM) else ""
        super().__init__(f"{where}: {msg} (status {code})" + (f" [{detail}]" if detail else ""))
        self.code = code


def _check(code: int, where: str):
    if code != HP_OK:
        raise HelmpreError(code, where)


def _host(a, shape):
    if a is None:
        return None
    arr = np.ascontiguousarray(np.asarray(a, dtype=np.float64))
    if arr.size != int(np.prod(shape)):
        raise ValueError(f"expected {int(np.prod(shape))} values, got {arr.size}")
    return arr


def _stream(stream):
    import torch
    s = torch.cuda.current_stream() if stream is None else stream
    return C.c_void_p(s.cuda_stream)


def _order_on(stream, *tensors):
    """Work the library enqueues on `stream` must see what the caller's current stream
    wrote to its tensors (an initial guess zeroed there, a right-hand side produced
    there): make `stream` wait for the current stream, and tell the caching allocator
    that the tensors are in use on `stream`."""
    import torch
    if stream is None:
        return
    cur = torch.cuda.current_stream(stream.device)
    if stream.cuda_stream == cur.cuda_stream:
        return
    stream.wait_stream(cur)
    for t in tensors:
        t.record_stream(stream)


@dataclass
class SolveInfo:
    iters: int
    cycles: int
    rel_true_residual: float
    status: int
    rel_prec_residual: float = float("nan")   # the residual the stopping test used (left: preconditioned)


class Plan:
    """Preconditioner plan: media, nodes, tables and workspace on the GPU.

    shape: grid points per axis (2 or 3 axes; each an even product of 2, 3 and 5 from 8
    to 4800, see hp_plan_create); length: side L.
    c, a, zeta: host arrays of that shape (a and zeta optional).
    precision: "fp64" (complex128 apply/matvec) or "mixed" (complex64 apply/matvec,
    FP64 orthogonalisation and residuals in solve).
    """

    def __init__(self, shape, omega, c, a=None, zeta=None, *, length=1.0, c0=1.0, m_real=8,
                 m_layer=3, symbol="continuous", precision="fp64", a_floor=0.0, max_nrhs=1,
                 nodes_real=None, nodes_zeta=None, a_nodes=None, stream=None, interp_order=1, m_damp=0,
                 layer_tensor=False):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("helmpre needs a ROCm GPU (torch.cuda.is_available() is False)")
        lib = load_library()
        self.shape = tuple(int(s) for s in shape)
        self.dim = len(self.shape)
        self.precision = precision
        self.npts = int(np.prod(self.shape))
        g = HpGrid()
        g.dim = self.dim
        for k, n in enumerate(self.shape):
            g.n[k] = n
            g.len[k] = float(length)
        self._grid = g
        keep = [_host(c, self.shape), _host(a, self.shape), _host(zeta, self.shape)]
        nr = None if nodes_real is None else np.ascontiguousarray(nodes_real, dtype=np.float64)
        nz = None if nodes_zeta is None else np.ascontiguousarray(nodes_zeta, dtype=np.float64)
        an = None if a_nodes is None else np.ascontiguousarray(a_nodes, dtype=np.float64)
        o = HpPlanOpts()
        o.m_real = int(m_real if nr is None else nr.size)
        o.m_layer = int(m_layer if nz is None else nz.size)
        o.nodes_real = None if nr is None else nr.ctypes.data
        o.nodes_zeta = None if nz is None else nz.ctypes.data
        o.a_nodes = None if an is None else an.ctypes.data
        o.a_floor = float(a_floor)
        o.symbol = SYMBOLS[symbol]
        o.precision = PRECISIONS[precision]
        o.max_nrhs = int(max_nrhs)
        o.interp_order = int(interp_order)
        o.m_damp = int(m_damp)
        o.layer_tensor = int(bool(layer_tensor))
        self._opts = o
        lay = HpLayer()
        lay.zeta = None if keep[2] is None else keep[2].ctypes.data
        lay.c0 = float(c0)
        h = C.c_void_p()
        code = lib.hp_plan_create(C.byref(h), C.byref(g), float(omega), keep[0].ctypes.data,
                                  None if keep[1] is None else keep[1].ctypes.data, C.byref(lay),
                                  C.byref(o), _stream(stream))
        _check(code, "hp_plan_create")
        self._h = h
        self.omega = float(omega)

    # dtype of apply / matvec fields
    @property
    def field_dtype(self):
        import torch
        return torch.complex128 if self.precision == "fp64" else torch.complex64

    def info(self) -> dict:
        pi = HpPlanInfo()
        _check(load_library().hp_plan_query(self._h, C.byref(pi)), "hp_plan_query")
        K = pi.K
        return {"K": K, "M": pi.M, "Mt": pi.Mt, "mo": pi.mo, "cmin": pi.cmin, "cmax": pi.cmax,
                "zeta_max": pi.zeta_max, "cnode": np.array(pi.cnode[:pi.M]),
                "znode": np.array(pi.znode[:pi.Mt + 1]), "ahat": np.array(pi.ahat[:K]),
                "gamma": np.array(pi.gamma_re[:K]) + 1j * np.array(pi.gamma_im[:K]),
                "workspace_bytes": int(pi.workspace_bytes), "interp_order": int(pi.interp_order),
                "m_damp": int(pi.m_damp), "layer_tensor": int(pi.layer_tensor),
                "anode": np.array(pi.anode[:(pi.K // pi.M if pi.layer_tensor else pi.m_damp)]),
                "tune": [tuple(int(x) for x in pi.tune[k]) for k in range(5)]}

    def _fields(self, x, dtype, name):
        import torch
        if not isinstance(x, torch.Tensor) or not x.is_cuda:
            raise TypeError(f"{name} must be a CUDA/HIP tensor")
        if x.dtype != dtype:
            raise TypeError(f"{name} must be {dtype}, got {x.dtype}")
        if not x.is_contiguous():
            raise ValueError(f"{name} must be contiguous")
        if tuple(x.shape[-self.dim:]) != self.shape:
            raise ValueError(f"{name} has shape {tuple(x.shape)}, grid is {self.shape}")
        return x.numel() // self.npts

    def _same_count(self, nr, x, dtype, name):
        """Check that the output/guess tensor x holds exactly nr fields (the library
        writes nr fields into it)."""
        n = self._fields(x, dtype, name)
        if n != nr:
            raise ValueError(f"{name} holds {n} fields, the input {nr}")
        return n

    def apply(self, v, out=None, stream=None):
        """u = Q_M v for one field or a batch [nrhs, *shape]."""
        import torch
        nr = self._fields(v, self.field_dtype, "v")
        u = torch.empty_like(v) if out is None else out
        self._same_count(nr, u, self.field_dtype, "out")
        _order_on(stream, v, u)
        _check(load_library().hp_apply_precond(self._h, C.c_void_p(v.data_ptr()), C.c_void_p(u.data_ptr()),
                                               nr, _stream(stream)), "hp_apply_precond")
        return u

    def apply_static(self, v, out=None, stream=None):
        """u = Q_M v through hp_apply_precond_static: the library's static device workspace
        (HP_STATIC_SCRATCH_BYTES per GPU) instead of the plan's; the C call allocates
        nothing (pass `out` to allocate nothing here either).  Calls on one GPU must not
        overlap."""
        import torch
        nr = self._fields(v, self.field_dtype, "v")
        u = torch.empty_like(v) if out is None else out
        self._same_count(nr, u, self.field_dtype, "out")
        _order_on(stream, v, u)
        lib = load_library()
        code = lib.hp_apply_precond_static(self._h, C.c_void_p(v.data_ptr()), C.c_void_p(u.data_ptr()), nr,
                                           _stream(stream))
        if code != HP_OK:   # the sizes of a refused call are in hp_last_error
            raise HelmpreError(code, "hp_apply_precond_static: " + lib.hp_last_error().decode())
        return u

    def matvec(self, u, out=None, stream=None):
        """y = P_N u for one field or a batch."""
        import torch
        nr = self._fields(u, self.field_dtype, "u")
        y = torch.empty_like(u) if out is None else out
        self._same_count(nr, y, self.field_dtype, "out")
        _order_on(stream, u, y)
        _check(load_library().hp_matvec(self._h, C.c_void_p(u.data_ptr()), C.c_void_p(y.data_ptr()), nr,
                                        _stream(stream)), "hp_matvec")
        return y

    def solve(self, f, x=None, *, restart=30, max_cycles=200, rtol=1e-8, stream=None, raise_on_fail=False,
              side="right"):
        """Restarted GMRES preconditioned by Q_M on the right (default) or left, or plain
        (side="none").  f (and x) complex128; returns (x, [SolveInfo])."""
        import torch
        nr = self._fields(f, torch.complex128, "f")
        if x is None:
            x = torch.zeros_like(f)
        self._same_count(nr, x, torch.complex128, "x")
        _order_on(stream, f, x)
        o = HpSolveOpts(int(restart), int(max_cycles), float(rtol), SIDES[side])
        infos = (HpSolveInfo * nr)()
        code = load_library().hp_solve(self._h, C.c_void_p(f.data_ptr()), C.c_void_p(x.data_ptr()), nr,
                                       C.byref(o), infos, _stream(stream))
        # per right-hand-side outcomes (not converged, non-finite) are in the infos
        if code not in (HP_OK, HP_E_NOT_CONVERGED, HP_E_NONFINITE) or (raise_on_fail and code != HP_OK):
            raise HelmpreError(code, "hp_solve")
        return x, [SolveInfo(i.iters, i.cycles, i.rel_true_residual, i.status, i.rel_prec_residual) for i in infos]

    def arnoldi(self, v0, m, side="left", stream=None):
        """m Arnoldi steps of Q P_N (left), P_N Q (right), P_N (none), (Q P_N)^{-1}
        (left_inverse) or P_N^{-1} (none_inverse) from v0 (complex128, one field,
        normalised); returns (H (m+1, m) complex128 numpy array, steps)."""
        import torch
        nr = self._fields(v0, torch.complex128, "v0")
        if nr != 1:
            raise ValueError("arnoldi takes one field")
        H = np.zeros((m + 1, m), dtype=np.complex128)
        steps = C.c_int(0)
        _check(load_library().hp_arnoldi(self._h, C.c_void_p(v0.data_ptr()), int(m), ARNOLDI_OPS[side],
                                         C.c_void_p(H.ctypes.data), C.byref(steps), _stream(stream)), "hp_arnoldi")
        return H, steps.value

    def autotune(self, stream=None):
        """Pick the fastest run-time choices of the transform passes (see hp_plan_autotune);
        returns (apply ms before, apply ms after)."""
        b, a = C.c_double(0.0), C.c_double(0.0)
        _check(load_library().hp_plan_autotune(self._h, C.byref(b), C.byref(a), _stream(stream)), "hp_plan_autotune")
        return b.value, a.value

    def arnoldi_vector(self, y, out=None, stream=None):
        """V_k y from the basis of the last arnoldi() on this plan (y: k complex numbers)."""
        import torch
        y = np.ascontiguousarray(y, dtype=np.complex128)
        if out is None:
            out = torch.empty(self.shape, dtype=torch.complex128, device="cuda")
        self._same_count(1, out, torch.complex128, "out")
        _check(load_library().hp_arnoldi_vector(self._h, C.c_void_p(y.ctypes.data), int(y.size),
                                                C.c_void_p(out.data_ptr()), _stream(stream)), "hp_arnoldi_vector")
        return out

    def extreme_eigenvalue(self, v0, smallest=False, side="left", m=64, max_restarts=20, tol=1e-6,
                           stream=None):
        """Eigenvalue of largest (or smallest) modulus of Q P_N / P_N Q / P_N by restarted
        Arnoldi; returns (lambda, relative residual, Arnoldi runs, converged)."""
        import torch
        if self._fields(v0, torch.complex128, "v0") != 1:
            raise ValueError("extreme_eigenvalue takes one field")
        lam = np.zeros(1, dtype=np.complex128)
        rr = C.c_double(0.0)
        runs = C.c_int(0)
        code = load_library().hp_extreme_eigenvalue(self._h, C.c_void_p(v0.data_ptr()), int(m), SIDES[side],
                                                    int(bool(smallest)), int(max_restarts), float(tol),
                                                    C.c_void_p(lam.ctypes.data), C.byref(rr), C.byref(runs),
                                                    _stream(stream))
        if code not in (0, 8):
            _check(code, "hp_extreme_eigenvalue")
        return complex(lam[0]), rr.value, runs.value, code == 0

    def spectral_cond(self, v0, side="left", m=64, max_restarts=20, tol=1e-6, stream=None):
        """Spectral condition number of Eqn. Cond, max |lambda| / min |lambda|, of the
        operator of `side`; returns (cond, details dict)."""
        hi = self.extreme_eigenvalue(v0, False, side, m, max_restarts, tol, stream)
        lo = self.extreme_eigenvalue(v0, True, side, m, max_restarts, tol, stream)
        det = {"max": hi[0], "min": lo[0], "max_rel_resid": hi[1], "min_rel_resid": lo[1],
               "runs": hi[2] + lo[2], "converged": hi[3] and lo[3]}
        return abs(hi[0]) / abs(lo[0]), det

    def profile_apply(self, v, out=None, reps=20, stream=None):
        """Event-timed applies: (ms per launch of the 5 pass slots, algorithmic bytes per pass)."""
        import torch
        nr = self._fields(v, self.field_dtype, "v")
        u = torch.empty_like(v) if out is None else out
        self._same_count(nr, u, self.field_dtype, "out")
        ms = (C.c_double * 5)()
        by = (C.c_double * 5)()
        _check(load_library().hp_profile_apply(self._h, C.c_void_p(v.data_ptr()), C.c_void_p(u.data_ptr()), nr,
                                               int(reps), ms, by, _stream(stream)), "hp_profile_apply")
        return list(ms), list(by)

    def time_pass(self, slot):
        """Record the start and end of every later launch of pass `slot` (0..4 as in
        profile_apply; None: off) in HIP events (hp_plan_time_pass); read them with pass_times()."""
        _check(load_library().hp_plan_time_pass(self._h, -1 if slot is None else int(slot)), "hp_plan_time_pass")

    def pass_times(self):
        """Milliseconds of each launch recorded since time_pass() or the last read, in order."""
        cap = 1 << 16                       # the most launches recorded per read
        ms = (C.c_double * cap)()
        n = C.c_int(0)
        _check(load_library().hp_plan_pass_times(self._h, ms, cap, C.byref(n)), "hp_plan_pass_times")
        return list(ms[:min(n.value, cap)])

    def close(self):
        if getattr(self, "_h", None):
            load_library().hp_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Solver:
    """Resumable restarted-GMRES solve on one stream (hp_solver_*): start(), then
    advance() without blocking until finished, then result().  The Krylov state
    stays on the GPU."""

    def __init__(self, plan, nrhs=1, *, restart=30, max_cycles=200, rtol=1e-8, side="right"):
        self.plan = plan
        self.nrhs = int(nrhs)
        self._opts = HpSolveOpts(int(restart), int(max_cycles), float(rtol), SIDES[side])
        h = C.c_void_p()
        _check(load_library().hp_solver_create(C.byref(h), plan._h, self.nrhs, C.byref(self._opts)),
               "hp_solver_create")
        self._h = h
        self._keep = None

    def start(self, f, x=None, stream=None):
        import torch
        nr = self.plan._fields(f, torch.complex128, "f")
        if nr != self.nrhs:
            raise ValueError(f"f holds {nr} right-hand sides, solver was made for {self.nrhs}")
        if x is None:
            x = torch.zeros_like(f)
        self.plan._same_count(nr, x, torch.complex128, "x")
        _order_on(stream, f, x)
        self._keep = (f, x, stream)
        _check(load_library().hp_solver_start(self._h, C.c_void_p(f.data_ptr()), C.c_void_p(x.data_ptr()),
                                              _stream(stream)), "hp_solver_start")
        return x

    def advance(self, max_steps=4):
        done = C.c_int(0)
        _check(load_library().hp_solver_advance(self._h, int(max_steps), C.byref(done)), "hp_solver_advance")
        return bool(done.value)

    def result(self):
        infos = (HpSolveInfo * self.nrhs)()
        code = load_library().hp_solver_wait(self._h, infos)
        if code not in (HP_OK, HP_E_NOT_CONVERGED, HP_E_NONFINITE):
            raise HelmpreError(code, "hp_solver_wait")
        return self._keep[1], [SolveInfo(i.iters, i.cycles, i.rel_true_residual, i.status, i.rel_prec_residual) for i in infos]

    def close(self):
        if getattr(self, "_h", None):
            load_library().hp_solver_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def advance_group(solvers, max_steps=4):
    """Advance several started Solver sessions together (hp_solver_advance_group): each
    round takes the next step of every one that is ready, those the grouped kernels take
    in one launch per pass.  All must have been started on the same stream.  Returns the
    list of finished flags."""
    n = len(solvers)
    if n == 0:
        return []
    hs = (C.c_void_p * n)(*[s._h for s in solvers])
    fin = (C.c_int * n)()
    _check(load_library().hp_solver_advance_group(hs, n, int(max_steps), fin), "hp_solver_advance_group")
    return [bool(v) for v in fin]


def ritz_values(H, steps, harmonic=False):
    """Ritz (harmonic=False) or harmonic Ritz values of the leading steps x steps block of
    an Arnoldi Hessenberg matrix H ((m+1, m) complex128, as Plan.arnoldi returns it)."""
    H = np.ascontiguousarray(H, dtype=np.complex128)
    m = H.shape[1]
    if H.shape != (m + 1, m):
        raise ValueError("H must be (m+1, m)")
    theta = np.zeros(int(steps), dtype=np.complex128)
    _check(load_library().hp_ritz_values(C.c_void_p(H.ctypes.data), int(m), int(steps), int(bool(harmonic)),
                                         C.c_void_p(theta.ctypes.data), None, None), "hp_ritz_values")
    return theta


def ritz_pairs(H, steps, harmonic=False):
    """(theta, Y, resid): Ritz or harmonic Ritz values, unit vectors y_i (rows of Y) and the
    residual norms ||A V y_i - theta_i V y_i|| of the Arnoldi relation."""
    H = np.ascontiguousarray(H, dtype=np.complex128)
    m = H.shape[1]
    if H.shape != (m + 1, m):
        raise ValueError("H must be (m+1, m)")
    k = int(steps)
    theta = np.zeros(k, dtype=np.complex128)
    Y = np.zeros((k, k), dtype=np.complex128)
    res = np.zeros(k, dtype=np.float64)
    _check(load_library().hp_ritz_values(C.c_void_p(H.ctypes.data), int(m), k, int(bool(harmonic)),
                                         C.c_void_p(theta.ctypes.data), C.c_void_p(Y.ctypes.data),
                                         res.ctypes.data_as(C.POINTER(C.c_double))), "hp_ritz_values")
    return theta, Y, res


def cond_estimate(H, steps):
    """(max |Ritz value|, min |harmonic Ritz value|, their ratio): an estimate of the
    spectral condition number of Eqn. Cond from one Arnoldi run (both ends approached
    from inside the spectrum)."""
    hi = float(np.abs(ritz_values(H, steps)).max())
    lo = float(np.abs(ritz_values(H, steps, harmonic=True)).min())
    return hi, lo, hi / lo


def workspace_bytes(shape, precision, K, nrhs=1, restart=30):
    """Device bytes a plan plus one solver of nrhs right-hand sides hold (admission by footprint)."""
    lib = load_library()
    g = HpGrid()
    g.dim = len(shape)
    for k, n in enumerate(shape):
        g.n[k] = int(n)
        g.len[k] = 1.0
    o = HpPlanOpts()
    o.precision = PRECISIONS[precision]
    o.max_nrhs = int(nrhs)
    return int(lib.hp_plan_workspace_bytes(C.byref(g), C.byref(o), int(K))) + \
        int(lib.hp_solve_workspace_bytes(C.byref(g), int(restart), int(nrhs)))


def plan_from_workload(w, **over):
    """Plan for a synthetic workload from paper_2409_16172_amd.inputs."""
    kw = dict(length=w.length, c0=w.c0, m_real=w.m_real, m_layer=w.m_layer, a_floor=w.a_floor,
              precision=w.precision, max_nrhs=w.f.shape[0])
    kw.update(over)
    return Plan(w.shape, w.omega, w.c, w.a, w.zeta, **kw)
