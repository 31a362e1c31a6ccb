"""Pins of the oracle's dL/dV (not gpu): central finite differences of L
evaluated by dense eigh, Sternheimer vs dense double sum, the shift
invariance sum_s dL/dV_s = sum_i g_i, Hellmann-Feynman at w = 0."""
import numpy as np
import pytest

from oracle import grad, stencil
from paper_1407_7506_amd import inputs as I


def setup(kpt, N=6, k=5, seed=3):
    V = I.gaussian_wells(N, 0.5, 2, seed)
    H = stencil.assemble_h(V, N, 0.5, 2, kpt)
    lam, X = np.linalg.eigh(H)
    return V, lam, X, N, k


@pytest.mark.parametrize("kpt", [(0.0, 0.0, 0.0), (0.3, 0.0, 0.0)])
def test_sternheimer_matches_dense_and_fd(kpt):
    V, lam, X, N, k = setup(kpt)
    rng = np.random.default_rng(1)
    g = rng.standard_normal(k)
    w = rng.standard_normal(N ** 3)
    dg = grad.dense_grad(lam, X, k, g, w)
    A = lambda Y: stencil.apply_h(Y, V, N, 0.5, 2, kpt)
    sg, it, rel = grad.sternheimer_grad(A, stencil.diag_h(V, 0.5, 2), X[:, :k], lam[:k], g, w, tol=1e-13)
    assert np.abs(sg - dg).max() <= 1e-10 * np.abs(dg).max()

    def L(Vv):
        l, Y = np.linalg.eigh(stencil.assemble_h(Vv, N, 0.5, 2, kpt))
        return grad.loss(l[:k], Y[:, :k], g, w)

    eps = 1e-5
    for d in I.unit_directions(N ** 3, 4, 2):
        fd = (L(V + eps * d) - L(V - eps * d)) / (2 * eps)
        assert abs(fd - dg @ d) <= 1e-6 * max(1.0, abs(fd))


def test_shift_invariance_and_hellmann_feynman():
    V, lam, X, N, k = setup((0.0, 0.0, 0.0))
    g = np.arange(1.0, k + 1)
    w = np.random.default_rng(4).standard_normal(N ** 3)
    dg = grad.dense_grad(lam, X, k, g, w)
    assert abs(dg.sum() - g.sum()) < 1e-10
    hf = grad.dense_grad(lam, X, k, g, None)
    np.testing.assert_allclose(hf, (X[:, :k] ** 2) @ g, atol=1e-14)
    np.testing.assert_allclose(grad.dense_grad(lam, X, k, g, np.zeros(N ** 3)), hf, atol=1e-14)
