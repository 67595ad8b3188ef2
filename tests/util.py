"""Small helpers shared by the tests (no method arithmetic)."""
import numpy as np


def rel(a, b):
    """||a - b|| / ||b|| over all entries (2-norm)."""
    a = np.asarray(a)
    b = np.asarray(b)
    nb = np.linalg.norm(b.ravel())
    return np.linalg.norm((a - b).ravel()) / (nb if nb > 0 else 1.0)


def rel_per_rhs(a, b):
    return np.array([rel(x, y) for x, y in zip(a, b)])
