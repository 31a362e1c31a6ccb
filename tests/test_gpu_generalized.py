"""GPU parity of the generalized problem H x = lambda B x (section 1: solved
without factoring B; B diagonal and positive here) against the oracle with the
same B and against scipy's eigh of the dense pencil, through the C ABI."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from oracle import brute, ppcg_ref, stencil  # noqa: E402
from paper_1407_7506_amd import binding as B  # noqa: E402
from paper_1407_7506_amd import inputs as I  # noqa: E402

MAX_IT = 4000


def say(*a):
    print(*a, flush=True)


def dev(a):
    return torch.tensor(np.ascontiguousarray(a), device="cuda")


def solve_both(p, b, handle_kw=None, oracle_kw=None):
    g = p.grid
    h = B.Handle("fp64", max_iter=MAX_IT, **(handle_kw or {}))
    lam, X, info = h.solve(dev(p.V), g.N, p.k, p.q, p.tol, p.rr_period, dev(p.start()), order=g.order,
                           kpt=g.kpt, B=dev(b))
    A = lambda Y: stencil.apply_h(Y, p.V, g.N, g.h, g.order, g.kpt)
    T = 1.0 / stencil.diag_h(p.V, g.h, g.order)
    lo, Xo, io = ppcg_ref.ppcg(A, T, p.start(), p.k, p.q, p.tol, p.rr_period, bdiag=b, **(oracle_kw or {}))
    h.close()
    return lam.cpu().numpy(), X.cpu().numpy(), info, lo, io


CASES = [dict(N=8, k=12, q=4, order=4), dict(N=10, k=20, q=4, order=2, kpt=(0.7, 0.0, 0.0)),
         dict(N=16, k=120, q=8, order=4),       # K = 128: B-weighted Grams on the LDS kernel
         dict(N=10, k=16, q=16, order=2, nbuf=16)]


@pytest.mark.parametrize("case", CASES, ids=lambda c: "-".join(f"{k}{v}" for k, v in c.items()))
def test_generalized_matches_oracle_and_pencil(case):
    p = I.small_problem(tol=1e-9, **case)
    g = p.grid
    b = I.mass_weights(g.N, g.h, 17)
    kw = {"nbuf": p.nbuf} if "nbuf" in case else {}
    lam, X, info, lo, io = solve_both(p, b, kw)
    ref = brute.lowest_values_gen(p.V, g.N, g.h, g.order, p.k, b, g.kpt)
    scale = np.abs(ref).max()
    say(p.name, "iters gpu/oracle", info["iters"], io.iters, "err vs oracle", np.abs(lam - lo).max() / scale,
        "vs pencil", np.abs(lam - ref).max() / scale, "orth_err", info["orth_err"])
    assert np.abs(lam - lo).max() / scale <= 1e-9
    assert np.abs(lam - ref).max() / scale <= 1e-9
    np.testing.assert_allclose(X.conj().T @ (b[:, None] * X), np.eye(p.k), atol=1e-11)
    R = stencil.apply_h(X, p.V, g.N, g.h, g.order, g.kpt) - (b[:, None] * X) * lam[None, :]
    assert np.linalg.norm(R) / np.linalg.norm(lam) <= 1e-9 * 1.001
    assert info["orth_err"] <= 1e-11 and info["resid_final"] <= 1e-9


def test_generalized_with_taylor_policy():
    p = I.small_problem(N=10, k=20, q=4, order=4, tol=1e-9)
    b = I.mass_weights(p.grid.N, p.grid.h, 18)
    lam, X, info, lo, io = solve_both(p, b, {"orth": "taylor"}, {"orth": "taylor"})
    say("generalized taylor: gpu taylor/skip", info["n_taylor"], info["n_orth_skip"], "oracle", io.n_taylor,
        io.n_orth_skip)
    assert np.abs(lam - lo).max() / np.abs(lo).max() <= 1e-9


def test_generalized_refusals():
    p = I.small_problem(N=8, k=12, q=4, order=2, tol=1e-8)
    g = p.grid
    b = I.mass_weights(g.N, g.h, 19)
    hm = B.Handle("mixed", max_iter=MAX_IT)
    with pytest.raises(B.PPCGError) as e:
        hm.solve(dev(p.V), g.N, p.k, p.q, p.tol, 5, dev(p.start()), B=dev(b))
    assert e.value.status == "PPCG_EINVAL"
    h = B.Handle("fp64", max_iter=MAX_IT)
    bad = b.copy()
    bad[7] = -0.1
    with pytest.raises(B.PPCGError) as e:
        h.solve(dev(p.V), g.N, p.k, p.q, p.tol, 5, dev(p.start()), B=dev(bad))
    assert e.value.status == "PPCG_ENOTHPD"
    h.solve(dev(p.V), g.N, p.k, p.q, p.tol, 5, dev(p.start()), B=dev(b))
    with pytest.raises(B.PPCGError) as e:
        h.grad(dev(np.ones(p.k)))
    assert e.value.status == "PPCG_EINVAL"
    h.close()
    hm.close()
