"""Dense brute force: every eigenpair of the assembled H by numpy.linalg.eigh
(oracle; test infrastructure).  Feasible for n up to a few thousand (the
16^3 workload assembles to a 4096 x 4096 matrix).

Pin: plane-wave closed form of the discrete Laplacian spectrum at V = 0
(tests/test_oracle_stencil.py).
"""
from __future__ import annotations

import numpy as np

from .stencil import assemble_h


def lowest(V, N, h, order, k, kpt=(0.0, 0.0, 0.0)):
    """(lam[:k], X[:, :k], lam_all) of H, ascending."""
    H = assemble_h(V, N, h, order, kpt)
    lam, X = np.linalg.eigh(H)
    return lam[:k], X[:, :k], lam


def lowest_values(V, N, h, order, k, kpt=(0.0, 0.0, 0.0)):
    """The k smallest eigenvalues of H (values only, numpy.linalg.eigvalsh)."""
    return np.linalg.eigvalsh(assemble_h(V, N, h, order, kpt))[:k]


def lowest_values_gen(V, N, h, order, k, b, kpt=(0.0, 0.0, 0.0)):
    """The k smallest eigenvalues of H x = lambda diag(b) x (scipy.linalg.eigh
    of the pencil, values only)."""
    import scipy.linalg as sla
    H = assemble_h(V, N, h, order, kpt)
    return sla.eigh(H, np.diag(np.asarray(b, dtype=np.float64)), eigvals_only=True)[:k]
