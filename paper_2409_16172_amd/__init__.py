"""MI355X (gfx950) implementation of the interpolated pseudodifferential
preconditioner for the variable-media Helmholtz equation (Acosta, Khajah,
Palacios, arXiv 2409.16172): HIP kernels behind a C ABI (libhelmpre.so), with a
thin ctypes binding.  `inputs` holds the seeded synthetic workloads."""
from . import inputs  # noqa: F401

__all__ = ["inputs", "Plan", "load_library", "plan_from_workload", "HelmpreError"]


def __getattr__(name):
    if name in ("Plan", "load_library", "plan_from_workload", "HelmpreError", "SolveInfo"):
        from . import binding
        return getattr(binding, name)
    raise AttributeError(name)
