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
    C, th, used_p, _, _ = dense.block_pencil(A, B, nx, True, _allow_backtrack=False)
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
    C, th, _, _, _ = dense.block_pencil(A, B, 1, False)
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
    C, th, used_p, back, dropped = dense.block_pencil(A, B, q, True)
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


# --- Theorem 1 indicator and the Theorem 2 backtrack (section 3) -----------------------------

def _pencil_from_operator(cplx, p_low, rng, q=2, n=40):
    """S = [X, W, P] from the eigenbasis Q of a Hermitian H = Q diag(lam) Q^H.
    X, W are orthonormal combinations of eigenvectors 10..13 (so x^H H w != 0);
    P spans eigenvectors 0..q-1 with a non-orthonormal basis, and their
    eigenvalues are ``p_low`` (below everything X and W reach when all are
    low, or only one of them below when p_low has a large second entry)."""
    Z = rng.standard_normal((n, n)) + (1j * rng.standard_normal((n, n)) if cplx else 0)
    Q, _ = np.linalg.qr(Z)
    lam = np.linspace(1.0, 5.0, n)
    lam[:q] = p_low
    H = (Q * lam) @ Q.conj().T
    Y = rng.standard_normal((4, 4)) + (1j * rng.standard_normal((4, 4)) if cplx else 0)
    Y, _ = np.linalg.qr(Y)
    X = Q[:, 10:14] @ Y[:, :q]
    W = Q[:, 10:14] @ Y[:, q:2 * q] * np.array([0.3, 2.0])[None, :q]
    Rp = rng.standard_normal((q, q)) + 3 * np.eye(q)
    P = Q[:, :q] @ Rp
    S = np.concatenate([X, W, P], axis=1)
    return dense.sym(S.conj().T @ H @ S), dense.sym(S.conj().T @ S), S, H


@pytest.mark.parametrize("cplx", [False, True])
@pytest.mark.parametrize("p_low", [(-10.0, -9.0), (-10.0, 10.0)], ids=["CX-zero", "CX-rank1"])
def test_theorem1_singular_cx_backtracks(cplx, p_low):
    """C_X of the q lowest pairs of the full pencil is singular (P spans the
    lowest directions and is orthogonal to X): the block is solved again
    without P and the result is exactly the 2q x 2q solution, whose C_X is
    nonsingular (Theorem 2, x^H H w != 0)."""
    rng = np.random.default_rng(31 + cplx)
    q = 2
    A, B, S, H = _pencil_from_operator(cplx, np.array(p_low), rng, q)
    # premise: with P the q lowest Ritz vectors have a singular X part
    full = dense.block_pencil(A, B, q, True, _allow_backtrack=False)
    assert full.used_p
    assert np.linalg.svd(full.C[:q], compute_uv=False).min() < 1e-10
    r = dense.block_pencil(A, B, q, True)
    assert r.backtracked and not r.used_p
    nop = dense.block_pencil(A, B, q, False)
    np.testing.assert_array_equal(r.C, nop.C)
    np.testing.assert_array_equal(r.theta, nop.theta)
    assert np.all(r.C[2 * q:] == 0)
    # the no-P solution against the library: the 2q lowest of (S2^H H S2, S2^H S2)
    S2 = S[:, :2 * q]
    ref = sla.eigh(S2.conj().T @ H @ S2, S2.conj().T @ S2, eigvals_only=True)[:q]
    np.testing.assert_allclose(r.theta, ref, rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(r.C.conj().T @ B @ r.C, np.eye(q), atol=1e-11)
    assert np.linalg.svd(r.C[:q], compute_uv=False).min() > 1e-3   # Theorem 2: alpha != 0


@pytest.mark.parametrize("cplx", [False, True])
def test_theorem1_threshold_is_absolute_pivot(cplx):
    """A weak X-P coupling makes C_X small but nonsingular: kept with P at the
    default floor, solved without P once singular_tol exceeds the smallest
    Cholesky pivot of C_X^H C_X (whose scale is 1: C^H B C = I)."""
    rng = np.random.default_rng(41 + cplx)
    q = 2
    A, B, S, H = _pencil_from_operator(cplx, np.array([-10.0, -9.0]), rng, q)
    eps = 1e-2
    A = A.copy()
    A[0, 2 * q] += eps
    A[2 * q, 0] += eps
    A[1, 2 * q + 1] += eps
    A[2 * q + 1, 1] += eps
    r = dense.block_pencil(A, B, q, True)
    assert r.used_p and not r.backtracked
    Cx = r.C[:q]
    ev = np.linalg.eigvalsh(dense.sym(Cx.conj().T @ Cx))
    assert 1e-12 < ev.min() and ev.max() < 1e-2
    # the Cholesky pivots of a q x q Gram lie between its extreme eigenvalues
    r2 = dense.block_pencil(A, B, q, True, singular_tol=ev.max() * 2)
    assert r2.backtracked and not r2.used_p
    np.testing.assert_array_equal(r2.C, dense.block_pencil(A, B, q, False).C)
    r3 = dense.block_pencil(A, B, q, True, singular_tol=ev.min() / 2)
    assert r3.used_p and not r3.backtracked


@pytest.mark.parametrize("cplx", [False, True])
@pytest.mark.parametrize("size", [0.02, 0.1, 0.3])
def test_polar_taylor_against_exact_polar_factor(cplx, size):
    """Four Taylor terms of (I + Y)^{-1/2} against the polar factor computed
    from the eigendecomposition of X^H X, within the series' remainder bound
    (35/128) |Y|^4 / (1 - |Y|) (spectral norms; section 5.5)."""
    rng = np.random.default_rng(int(size * 100) + cplx)
    n, m = 300, 24
    Q, _ = np.linalg.qr(rng.standard_normal((n, m)) + (1j * rng.standard_normal((n, m)) if cplx else 0))
    E = rng.standard_normal((m, m)) + (1j * rng.standard_normal((m, m)) if cplx else 0)
    E = dense.sym(E)
    E *= size / np.linalg.norm(E, 2) / 2.5
    X = Q @ (np.eye(m) + E)                  # X^H X = (I + E)^2: |Y| about 2 |E|
    G = dense.sym(X.conj().T @ X)
    ev, U = np.linalg.eigh(G)
    exact = X @ (U * ev ** -0.5) @ U.conj().T
    y = np.linalg.norm(G - np.eye(m), 2)
    bound = 35 / 128 * y ** 4 / (1 - y)
    Xt = dense.polar_taylor(X, G)
    # X (T - (I+Y)^{-1/2}) has spectral norm <= |X|_2 * remainder
    err = np.linalg.norm(Xt - exact, 2)
    assert err <= bound * np.linalg.norm(X, 2) * 1.0001 + 1e-14
    assert err >= 1e-3 * bound          # the truncation is what is measured, not rounding
    np.testing.assert_allclose(exact.conj().T @ exact, np.eye(m), atol=1e-12)
