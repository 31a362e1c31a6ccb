"""Pins of the oracle's operator: plane-wave closed form, dense assembly,
Hermitian symmetry (not gpu)."""
import numpy as np
import pytest

from oracle import stencil


def symbol(theta, h, order):
    """Closed-form eigenvalue of -1/2 d^2/dx^2 (discrete) for e^{i theta x/h}."""
    if order == 2:
        return 0.5 * 4.0 * np.sin(theta / 2) ** 2 / h ** 2
    return 0.5 * (30.0 - 32.0 * np.cos(theta) + 2.0 * np.cos(2 * theta)) / (12.0 * h ** 2)


@pytest.mark.parametrize("order", [2, 4])
@pytest.mark.parametrize("kpt", [(0.0, 0.0, 0.0), (0.37, 0.0, 0.0), (0.2, -0.5, 0.9)])
def test_plane_waves_closed_form(order, kpt):
    N, h = 6, 0.5
    idx = np.arange(N)
    z, y, x = np.meshgrid(idx, idx, idx, indexing="ij")
    coords = [x.ravel(), y.ravel(), z.ravel()]
    rng = np.random.default_rng(0)
    for _ in range(5):
        m = rng.integers(0, N, size=3)
        th = 2 * np.pi * m / N
        u = np.exp(1j * (th[0] * coords[0] + th[1] * coords[1] + th[2] * coords[2]))
        lam = sum(symbol(th[d] + kpt[d] * h, h, order) for d in range(3))
        Hu = stencil.apply_h(u.astype(np.complex128), np.zeros(N ** 3), N, h, order, kpt)
        np.testing.assert_allclose(Hu, lam * u, atol=1e-12)


@pytest.mark.parametrize("order,N", [(2, 4), (2, 5), (4, 5), (4, 6)])
@pytest.mark.parametrize("kpt", [(0.0, 0.0, 0.0), (0.3, 0.1, -0.2)])
def test_matrix_free_matches_assembled(order, N, kpt):
    rng = np.random.default_rng(N + order)
    V = rng.standard_normal(N ** 3)
    H = stencil.assemble_h(V, N, 0.5, order, kpt)
    cplx = any(kpt)
    X = rng.standard_normal((N ** 3, 3)) + (1j * rng.standard_normal((N ** 3, 3)) if cplx else 0)
    np.testing.assert_allclose(stencil.apply_h(X, V, N, 0.5, order, kpt), H @ X, atol=1e-12)
    np.testing.assert_allclose(np.diag(H).real, stencil.diag_h(V, 0.5, order))
    np.testing.assert_allclose(H, H.conj().T, atol=0)


def test_hermitian_products():
    N = 7
    rng = np.random.default_rng(3)
    V = rng.standard_normal(N ** 3)
    kpt = (0.4, 0.0, 0.0)
    x = rng.standard_normal(N ** 3) + 1j * rng.standard_normal(N ** 3)
    y = rng.standard_normal(N ** 3) + 1j * rng.standard_normal(N ** 3)
    Hx = stencil.apply_h(x, V, N, 0.5, 4, kpt)
    Hy = stencil.apply_h(y, V, N, 0.5, 4, kpt)
    assert abs(np.vdot(y, Hx) - np.vdot(Hy, x)) < 1e-10 * abs(np.vdot(y, Hx))
