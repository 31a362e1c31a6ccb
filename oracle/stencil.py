"""Finite-difference Kohn-Sham operator H = -1/2 Lap_h + diag(V) on a periodic
N^3 grid, applied matrix-free with np.roll (oracle; test infrastructure).

The paper only needs products A x with a Hermitian A (statement of the
problem, section 1); its experiments use planewave Hamiltonians.  Here A is
a finite-difference operator:
  order 2: 7-point Laplacian, second difference (u(+1) - 2u + u(-1)) / h^2
           per direction;
  order 4: 13-point Laplacian, (-u(-2) + 16u(-1) - 30u + 16u(+1) - u(+2)) / (12 h^2)
           per direction.
A Bloch vector kappa enters in gauge (Peierls) form: the coupling from point r
to r + a*h*e_d carries the factor exp(i kappa_d a h), which keeps the operator
Hermitian and periodic.

Pins (tests/test_oracle_stencil.py): plane waves at V = 0 against the closed
form symbol, dense assembly against the matrix-free product, Hermitian
symmetry <y, Hx> = <Hy, x>.
"""
from __future__ import annotations

import numpy as np

# second-derivative stencil weights by offset, for -1/2 * d^2/dx^2 (h = 1)
_W2 = {0: 1.0, 1: -0.5}                       # 7-point: -1/2 * (1, -2, 1)
_W4 = {0: 1.25, 1: -2.0 / 3.0, 2: 1.0 / 24.0}  # 13-point: -1/2 * (-1,16,-30,16,-1)/12


def _weights(order: int) -> dict:
    if order == 2:
        return _W2
    if order == 4:
        return _W4
    raise ValueError("order must be 2 (7-point) or 4 (13-point)")


def diag_h(V: np.ndarray, h: float, order: int) -> np.ndarray:
    """Diagonal of H: 3 * w0 / h^2 + V (the Bloch phase does not touch it)."""
    return 3.0 * _weights(order)[0] / (h * h) + np.asarray(V, dtype=np.float64)


def apply_h(X: np.ndarray, V: np.ndarray, N: int, h: float, order: int,
            kpt=(0.0, 0.0, 0.0)) -> np.ndarray:
    """H @ X for X of shape (n,) or (n, m), n = N^3, grid index i + N(j + N l)."""
    X = np.asarray(X)
    vec = X.ndim == 1
    Xm = X[:, None] if vec else X
    m = Xm.shape[1]
    complex_ = any(float(c) != 0.0 for c in kpt) or np.iscomplexobj(Xm)
    dt = np.complex128 if complex_ else np.float64
    U = Xm.astype(dt, copy=False).reshape(N, N, N, m)   # axes: z, y, x, column
    w = _weights(order)
    inv_h2 = 1.0 / (h * h)
    Y = (3.0 * w[0] * inv_h2) * U + V.reshape(N, N, N, 1) * U
    axis_of = {0: 2, 1: 1, 2: 0}  # direction d -> array axis
    for d in range(3):
        ax = axis_of[d]
        for a, wa in w.items():
            if a == 0:
                continue
            # neighbour u(r + a e_d) is np.roll(U, -a, axis)
            ph = np.exp(1j * kpt[d] * a * h) if complex_ else 1.0
            Y = Y + (wa * inv_h2) * (ph * np.roll(U, -a, axis=ax) + np.conj(ph) * np.roll(U, a, axis=ax))
    Y = Y.reshape(N ** 3, m)
    if not complex_:
        Y = Y.real if np.iscomplexobj(Y) else Y
    return Y[:, 0] if vec else Y


def assemble_h(V: np.ndarray, N: int, h: float, order: int, kpt=(0.0, 0.0, 0.0)) -> np.ndarray:
    """Dense n x n matrix of H, built entry by entry from the stencil
    definition (independent of np.roll; for tiny grids only)."""
    n = N ** 3
    complex_ = any(float(c) != 0.0 for c in kpt)
    H = np.zeros((n, n), dtype=np.complex128 if complex_ else np.float64)
    w = _weights(order)
    inv_h2 = 1.0 / (h * h)
    for l in range(N):
        for j in range(N):
            for i in range(N):
                r = i + N * (j + N * l)
                H[r, r] += 3.0 * w[0] * inv_h2 + V[r]
                for a, wa in w.items():
                    if a == 0:
                        continue
                    for sgn in (1, -1):
                        off = sgn * a
                        for d in range(3):
                            c = [i, j, l]
                            c[d] = (c[d] + off) % N
                            s = c[0] + N * (c[1] + N * c[2])
                            val = wa * inv_h2
                            if complex_:
                                val = val * np.exp(1j * kpt[d] * off * h)
                            H[r, s] += val
    return H
