"""Pins of the oracle's small dense steps against library routines and closed
forms (not gpu)."""
import numpy as np
import pytest
import scipy.linalg as sla

from oracle import dense


def rand_pencil(nb, cplx, rng, cond=10.0):
    M = rng.standard_normal((nb, nb)) + (1j * rng.standard_normal((nb, nb)) if cplx else 0)
    A = dense.sym(M)
    Z = rng.standard_normal((nb, nb)) + (1j * rng.standard_normal((nb, nb)) if cplx else 0)
    Qz, _ = np.linalg.qr(Z)
    s = np.geomspace(1.0, 1.0 / cond, nb)
    B = dense.sym((Qz * s) @ Qz.conj().T)
    return A, B


@pytest.mark.parametrize("nb", [6, 24, 48, 96])
@pytest.mark.parametrize("cplx", [False, True])
def test_block_pencil_matches_scipy(nb, cplx):
    rng = np.random.default_rng(nb + cplx)
    A, B = rand_pencil(nb, cplx, rng)
    nx = nb // 3
    C, th, used_p = dense.block_pencil(A, B, nx, True, _allow_backtrack=False)
    ref = sla.eigh(A, B, eigvals_only=True)
    np.testing.assert_allclose(th, ref[:nx], rtol=1e-11, atol=1e-11)
    np.testing.assert_allclose(C.conj().T @ B @ C, np.eye(nx), atol=1e-11)
    np.testing.assert_allclose(A @ C, B @ C * th[None, :], atol=1e-10)


def test_two_by_two_closed_form():
    # 2 x 2 pencil in the proof of Theorem 2: [[a, b], [b, c]] vs diag(1, d) -- lowest root of
    # det(A - theta B) = 0:  d theta^2 - (a d + c) theta + (a c - b^2) = 0
    a, b, c, d = 0.7, 0.3, 2.5, 0.04
    A = np.array([[a, b], [b, c]])
    B = np.diag([1.0, d])
    C, th, _ = dense.block_pencil(A, B, 1, False)
    disc = (a * d + c) ** 2 - 4 * d * (a * c - b * b)
    root = ((a * d + c) - np.sqrt(disc)) / (2 * d)
    assert abs(th[0] - root) < 1e-13
    # Theorem 2: x^* A w = b != 0 implies alpha != 0
    assert abs(C[0, 0]) > 0


def test_block_pencil_drops_dependent_and_zero_columns():
    rng = np.random.default_rng(5)
    n, q = 200, 3
    X, _ = np.linalg.qr(rng.standard_normal((n, q)))
    W = rng.standard_normal((n, q))
    W -= X @ (X.T @ W)
    W[:, 1] = 0.0                          # a zero search direction
    P = W.copy()                           # P duplicates W: dependent columns
    H = dense.sym(rng.standard_normal((n, n)))
    S = np.concatenate([X, W, P], axis=1)
    A, B = S.T @ H @ S, S.T @ S
    C, th, used_p = dense.block_pencil(A, B, q, True)
    assert np.all(C[q + 1] == 0) and np.all(C[2 * q:] == 0)
    assert not used_p
    np.testing.assert_allclose(C.T @ B @ C, np.eye(q), atol=1e-10)
    # the kept span is [X, W0, W2]; its q lowest Ritz values
    S2 = np.concatenate([X, W[:, [0, 2]]], axis=1)
    ref = sla.eigh(S2.T @ H @ S2, S2.T @ S2, eigvals_only=True)[:q]
    np.testing.assert_allclose(th, ref, atol=1e-10)


@pytest.mark.parametrize("cplx", [False, True])
def test_cholqr(cplx):
    rng = np.random.default_rng(11)
    X = rng.standard_normal((300, 20)) + (1j * rng.standard_normal((300, 20)) if cplx else 0)
    Q, R = dense.cholqr(X)
    np.testing.assert_allclose(Q.conj().T @ Q, np.eye(20), atol=1e-12)
    np.testing.assert_allclose(Q @ R, X, atol=1e-12)
    assert np.allclose(R, np.triu(R))
    Xd = X.copy()
    Xd[:, 3] = Xd[:, 5]
    with pytest.raises(dense.RankError):
        dense.cholqr(Xd)


@pytest.mark.parametrize("cplx", [False, True])
def test_rayleigh_ritz(cplx):
    rng = np.random.default_rng(12)
    n, K = 120, 10
    H = dense.sym(rng.standard_normal((n, n)) + (1j * rng.standard_normal((n, n)) if cplx else 0))
    S = rng.standard_normal((n, K)) + (1j * rng.standard_normal((n, K)) if cplx else 0)
    X, lam, C = dense.rayleigh_ritz(S, H @ S)
    ref = sla.eigh(S.conj().T @ H @ S, S.conj().T @ S, eigvals_only=True)
    np.testing.assert_allclose(lam, ref, rtol=1e-11, atol=1e-11)
    np.testing.assert_allclose(X.conj().T @ X, np.eye(K), atol=1e-11)
    np.testing.assert_allclose(X.conj().T @ H @ X, np.diag(lam), atol=1e-10)
