"""Small dense steps of PPCG (oracle; test infrastructure).

  sym            Hermitian part (M + M^H)/2 of a computed Gram
  cholqr         Cholesky-QR: X^H X = R^H R, X <- X R^{-1} (section 5.5)
  polar_taylor   X (X^H X)^{-1/2} by four Taylor terms (section 5.5)
  block_pencil   the 3q x 3q (2q x 2q without P) projected problem of the block
                 update (section 5.1, with the projected problem of section 2);
                 C^H B C = I, the q lowest
  rayleigh_ritz  the full Rayleigh-Ritz over [X, X_lock] (Algorithm 3, RR branch)

Library primitives used as single steps: scipy.linalg.cholesky,
scipy.linalg.solve_triangular, numpy.linalg.eigh.

Readings where the paper is silent:
  * Computed Grams are replaced by their Hermitian part.
  * The block pencil is diagonally scaled (D = diag(B)^{-1/2}); W or P columns
    whose squared norm is below (1e-14)^2 times the largest X-column squared
    norm are dropped (zero search direction).  The scaled B is factored by a
    Cholesky that accepts columns in the order X, W, P and drops a column
    whose pivot falls below PIVOT_TOL (a direction that is numerically in the
    span of the columns already accepted).
  * Theorem 1 indicator in block form: if C_X of the kept eigenvectors is
    numerically singular (a Cholesky pivot of C_X^H C_X below PIVOT_TOL; the
    columns of C are B-orthonormal and X is orthonormal and orthogonal to W
    and P, so C_X^H C_X <= I and its scale is 1) and P was used, the block is
    solved again without P (the backtrack of Theorem 2).

Pins: tests/test_oracle_dense.py (scipy.linalg.eigh(A, B) on random pencils,
the closed-form 2 x 2 problem in the proof of Theorem 2, C^H B C = I, CholQR invariants).
"""
from __future__ import annotations

from typing import NamedTuple

import numpy as np
import scipy.linalg as sla

DROP_TOL = 1e-14      # relative norm below which a W/P column counts as zero
PIVOT_TOL = 1e-12     # Cholesky pivot (of a unit-diagonal matrix) floor


class RankError(RuntimeError):
    """Cholesky-QR or Rayleigh-Ritz met a numerically rank-deficient block."""


class PencilResult(NamedTuple):
    C: np.ndarray          # (rows of A, nx) coefficients, zero rows for dropped columns
    theta: np.ndarray      # the nx lowest Ritz values, ascending
    used_p: bool           # some P column took part in the returned solution
    backtracked: bool      # Theorem 1 test failed; solved again without P
    dropped: int           # W/P columns of the solved pencil left out as zero or dependent


def sym(M: np.ndarray) -> np.ndarray:
    return 0.5 * (M + M.conj().T)


def cholqr(X: np.ndarray, BX: np.ndarray | None = None):
    """Return (X R^{-1}, R) with R upper triangular, R^H R = sym(X^H X), or
    sym(X^H B X) when BX = B X is given (B-orthonormal result)."""
    G = sym(X.conj().T @ (X if BX is None else BX))
    try:
        R = sla.cholesky(G, lower=False)
    except np.linalg.LinAlgError as e:
        raise RankError(f"Cholesky-QR breakdown: {e}") from None
    # X R^{-1} = (R^{-T} X^T)^T, with R^T lower triangular (no conjugation)
    Q = sla.solve_triangular(R.T, X.T, lower=True).T
    return Q, R


def _greedy_cholesky(B: np.ndarray, order: list, tol: float):
    """Cholesky of B restricted to the columns accepted greedily in ``order``:
    column c is accepted when its pivot B_cc - sum_p |L_cp|^2 over accepted p
    is at least ``tol``.  Returns (accepted list, lower factor L)."""
    acc = []
    L = np.zeros((len(order), len(order)), dtype=B.dtype)
    for c in order:
        r = len(acc)
        row = np.zeros(r, dtype=B.dtype)
        for t, p in enumerate(acc):
            row[t] = (B[c, p] - np.dot(row[:t], L[t, :t].conj())) / L[t, t]
        piv = (B[c, c] - np.vdot(row, row)).real
        if piv >= tol:
            L[r, :r] = row
            L[r, r] = np.sqrt(piv)
            acc.append(c)
    nacc = len(acc)
    return acc, L[:nacc, :nacc]


def block_pencil(A: np.ndarray, B: np.ndarray, nx: int, has_p: bool, _allow_backtrack=True,
                 singular_tol: float = PIVOT_TOL):
    """Lowest nx eigenpairs of the projected pencil (A, B) of one sub-block
    S = [X_j, W_j, P_j] (columns 0..nx-1 are X_j, then nx W_j columns, then
    nx P_j columns when has_p).  Returns a PencilResult: C has shape
    (rows of A, nx), C^H B C = I on the kept rows and dropped rows are zero;
    backtracked is True when the Theorem 1 test found C_X singular (a
    Cholesky pivot of C_X^H C_X below singular_tol) and the block was solved
    again without P (Theorem 2)."""
    nb = A.shape[0]
    A = sym(A)
    B = sym(B)
    d = np.real(np.diag(B)).copy()
    xmax = max(d[:nx].max(), np.finfo(float).tiny)
    keep = []
    for c in range(nb):
        if c >= 2 * nx and not has_p:
            continue
        if c < nx or d[c] > (DROP_TOL ** 2) * xmax:
            keep.append(c)
    Dv = np.zeros(nb)
    Dv[keep] = 1.0 / np.sqrt(d[keep])
    Bs = Dv[:, None] * B * Dv[None, :]
    As = Dv[:, None] * A * Dv[None, :]
    acc, L = _greedy_cholesky(Bs, keep, PIVOT_TOL)
    if len(acc) < nx:
        raise RankError("block pencil has fewer independent columns than wanted pairs")
    Asub = As[np.ix_(acc, acc)]
    # M = L^{-1} A L^{-H}
    T = sla.solve_triangular(L, Asub, lower=True)
    M = sla.solve_triangular(L, T.conj().T, lower=True).conj().T
    theta, Y = np.linalg.eigh(sym(M))
    Cacc = sla.solve_triangular(L.conj().T, Y[:, :nx], lower=False)
    C = np.zeros((nb, nx), dtype=np.result_type(A.dtype, B.dtype, np.float64))
    C[acc, :] = Dv[acc, None] * Cacc
    used_p = has_p and any(c >= 2 * nx for c in acc)
    if used_p and _allow_backtrack:
        # C^H B C = I with X orthonormal and orthogonal to W, P gives
        # C_X^H C_X <= I: its pivots are compared with 1, not with its own
        # largest entry (a C_X that vanishes to rounding is singular too)
        Cx = C[:nx, :]
        G = sym(Cx.conj().T @ Cx)
        _, Lx = _greedy_cholesky(G, list(range(nx)), singular_tol)
        if Lx.shape[0] < nx:
            r = block_pencil(A, B, nx, False, _allow_backtrack=False)
            return PencilResult(r.C, r.theta, False, True, r.dropped)
    nfull = (3 if has_p else 2) * nx
    return PencilResult(C, theta[:nx], used_p, False, nfull - len(acc))


def polar_taylor(X: np.ndarray, G: np.ndarray) -> np.ndarray:
    """Nearly orthonormal X -> X (X^H X)^{-1/2}, the orthonormal factor of its
    polar decomposition, with (I + Y)^{-1/2} replaced by the first four terms
    of the Taylor series of (1 + y)^{-1/2}: I - Y/2 + 3 Y^2/8 - 5 Y^3/16,
    Y = G - I, G = sym(X^H X) (section 5.5).  The truncation error in the
    spectral norm is at most (35/128) |Y|^4 / (1 - |Y|) for |Y| < 1."""
    Y = sym(G) - np.eye(G.shape[0])
    Y2 = Y @ Y
    T = np.eye(G.shape[0]) - 0.5 * Y + 0.375 * Y2 - 0.3125 * (Y2 @ Y)
    return X @ T


def rayleigh_ritz(S: np.ndarray, AS: np.ndarray, BS: np.ndarray | None = None):
    """Ritz pairs of span(S): sym(S^H A S) C = sym(S^H B S) C Omega,
    C^H S^H B S C = I (B = I when BS is None), all columns, ascending.
    Returns (S C, Omega, C)."""
    SAS = sym(S.conj().T @ AS)
    SS = sym(S.conj().T @ (S if BS is None else BS))
    try:
        L = sla.cholesky(SS, lower=True)
    except np.linalg.LinAlgError as e:
        raise RankError(f"Rayleigh-Ritz Gram not positive definite: {e}") from None
    T = sla.solve_triangular(L, SAS, lower=True)
    M = sla.solve_triangular(L, T.conj().T, lower=True).conj().T
    lam, Y = np.linalg.eigh(sym(M))
    C = sla.solve_triangular(L.conj().T, Y, lower=False)
    return S @ C, lam, C
