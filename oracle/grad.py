"""dL/dV for L = sum_i g_i lambda_i + sum_r w_r rho_r, rho = sum_{i<=k} |x_i|^2
(oracle; test infrastructure).

The eigenvalue part is Hellmann-Feynman: d lambda_i / d V_s = |x_i(s)|^2 since
H depends on V through its diagonal.  The density part is first-order
perturbation theory of the occupied subspace: with Q = I - X X^H,
    d rho = 2 Re sum_i conj(x_i) * dx_i,  dx_i = -(Q (H - lambda_i) Q)^+ Q dH x_i,
so  dL/dV = sum_i g_i |x_i|^2 - 2 Re sum_i conj(z_i) * x_i  with z_i the
solution (orthogonal to X) of the projected Sternheimer system
    Q (H - lambda_i) Q z_i = Q (w * x_i).

sternheimer_grad  solves those systems by plain preconditioned CG, one
                  column per wanted pair (Jacobi preconditioner
                  1/(diag(H) - lambda_i), projected).
dense_grad        the same derivative from a full eigendecomposition (tiny
                  grids): sum over occupied i and empty j of
                  2 Re(conj(x_i(r)) x_j(r) conj(x_j(s)) x_i(s)) / (lambda_i - lambda_j).

Pins (tests/test_oracle_grad.py): central finite differences of L evaluated by
dense eigh, the two forms against each other, sum_s dL/dV_s = sum_i g_i
(rho is invariant under V -> V + c), and w = 0 giving Hellmann-Feynman.
"""
from __future__ import annotations

import numpy as np


def _proj(X, Y):
    return Y - X @ (X.conj().T @ Y)


def sternheimer_grad(apply_a, diag_h, X, lam, g_lam, w, tol=1e-12, max_iter=5000):
    """Returns (dL/dV (n,), CG iterations, final relative residual)."""
    X = np.asarray(X)
    lam = np.asarray(lam, dtype=np.float64)
    n, k = X.shape
    dens = np.real(X.conj() * X)
    out = dens @ np.asarray(g_lam, dtype=np.float64)
    if w is None:
        return out, 0, 0.0
    w = np.asarray(w, dtype=np.float64)
    Minv = diag_h[:, None] - lam[None, :]
    if np.any(Minv <= 0):
        Minv = np.ones_like(Minv)          # plain CG when the shift breaks positivity
    Minv = 1.0 / Minv
    b = _proj(X, w[:, None] * X)
    bn = np.sqrt(np.real(np.sum(b.conj() * b, axis=0)))
    bn[bn == 0] = 1.0
    z = np.zeros_like(b)
    r = b.copy()
    y = _proj(X, Minv * r)
    p = y.copy()
    rz = np.real(np.sum(r.conj() * y, axis=0))
    it = 0
    rel = np.sqrt(np.real(np.sum(r.conj() * r, axis=0))) / bn
    while it < max_iter and rel.max() > tol:
        Ap = _proj(X, apply_a(p) - p * lam[None, :])
        pAp = np.real(np.sum(p.conj() * Ap, axis=0))
        alpha = np.where(pAp > 0, rz / np.where(pAp > 0, pAp, 1.0), 0.0)
        z = z + p * alpha[None, :]
        r = r - Ap * alpha[None, :]
        y = _proj(X, Minv * r)
        rz_new = np.real(np.sum(r.conj() * y, axis=0))
        beta = np.where(rz > 0, rz_new / np.where(rz > 0, rz, 1.0), 0.0)
        p = y + p * beta[None, :]
        rz = rz_new
        it += 1
        rel = np.sqrt(np.real(np.sum(r.conj() * r, axis=0))) / bn
    out = out - 2.0 * np.real(np.sum(z.conj() * X, axis=1))
    return out, it, float(rel.max())


def dense_grad(lam_all, X_all, k, g_lam, w):
    """dL/dV from the full spectrum (lam_all ascending, X_all columns)."""
    Xo = X_all[:, :k]
    out = np.real(Xo.conj() * Xo) @ np.asarray(g_lam, dtype=np.float64)
    if w is None:
        return out
    Xe = X_all[:, k:]
    M = Xo.conj().T @ (np.asarray(w)[:, None] * Xe)          # k x (n-k): x_i^H diag(w) x_j
    dl = lam_all[:k, None] - lam_all[None, k:]                # lambda_i - lambda_j
    F = M / dl
    # sum_ij 2 Re( M_ij/(l_i-l_j) * conj(x_j(s)) x_i(s) )
    T = Xe.conj() @ F.T                                        # n x k : sum_j conj(x_j(s)) F_ij
    return out + 2.0 * np.real(np.sum(T * Xo, axis=1))


def loss(lam, X, g_lam, w):
    """L = sum g_i lambda_i + sum_r w_r rho_r."""
    rho = np.sum(np.real(X.conj() * X), axis=1)
    return float(np.dot(g_lam, lam) + (np.dot(w, rho) if w is not None else 0.0))
