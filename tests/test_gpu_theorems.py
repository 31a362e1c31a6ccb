"""GPU parity of the sub-block step's safeguards (section 5.1; Theorems 1-2
of section 3) and of the solver's boundary behaviour, through the C ABI.

* ppcg_block_pencils: the q lowest pairs of given 3q x 3q (2q x 2q) pencils
  against the oracle's block_pencil, including pencils whose C_X is singular
  (the re-solve without P of Theorem 2) and the singular_tol threshold.
* ppcg_solve on problems where the backtrack fires, where the locked set
  shrinks, and whose start block holds an exact eigenvector.
* the start block drawn on the device (X0 = NULL) and ppcg_start_block
  against the oracle's generator, the solve without a preconditioner
  (T = I), the persisted autotuner
  table, the per-iteration log, the stage times, and ppcg_grad's
  PPCG_ENOCONV."""
import math
import os

import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from oracle import brute, dense, ppcg_ref, rng, stencil  # noqa: E402
from paper_1407_7506_amd import binding as B  # noqa: E402
from paper_1407_7506_amd import inputs as I  # noqa: E402

MAX_IT = 4000


def say(*a):
    print(*a, flush=True)


def dev(a):
    return torch.tensor(np.ascontiguousarray(a), device="cuda")


@pytest.fixture(scope="module")
def h64():
    h = B.Handle("fp64", max_iter=MAX_IT)
    yield h
    h.close()


def rand_pencil(nb, cplx, rng, cond=10.0):
    M = rng.standard_normal((nb, nb)) + (1j * rng.standard_normal((nb, nb)) if cplx else 0)
    A = dense.sym(M)
    Z = rng.standard_normal((nb, nb)) + (1j * rng.standard_normal((nb, nb)) if cplx else 0)
    Qz, _ = np.linalg.qr(Z)
    s = np.geomspace(1.0, 1.0 / cond, nb)
    return A, dense.sym((Qz * s) @ Qz.conj().T)


def op_pencil(cplx, p_low, rng, q=2, n=40, eps=0.0):
    """S = [X, W, P] in the eigenbasis of H = Q diag(lam) Q^H: X and W mix
    eigenvectors 10..13, P spans eigenvectors 0..q-1 (eigenvalues p_low) with
    a non-orthonormal basis; eps couples x_t to p_t in A."""
    Z = rng.standard_normal((n, n)) + (1j * rng.standard_normal((n, n)) if cplx else 0)
    Q, _ = np.linalg.qr(Z)
    lam = np.linspace(1.0, 5.0, n)
    lam[:q] = p_low
    H = (Q * lam) @ Q.conj().T
    Y = rng.standard_normal((2 * q, 2 * q)) + (1j * rng.standard_normal((2 * q, 2 * q)) if cplx else 0)
    Y, _ = np.linalg.qr(Y)
    X = Q[:, 10:10 + 2 * q] @ Y[:, :q]
    W = Q[:, 10:10 + 2 * q] @ Y[:, q:] * np.linspace(0.3, 2.0, q)[None, :]
    P = Q[:, :q] @ (rng.standard_normal((q, q)) + 3 * np.eye(q))
    S = np.concatenate([X, W, P], axis=1)
    A = dense.sym(S.conj().T @ H @ S)
    for t in range(q):
        A[t, 2 * q + t] += eps
        A[2 * q + t, t] += eps
    return A, dense.sym(S.conj().T @ S)


def gpu_pencils(h, As, Bs, q, has_p, tol=1e-9):
    """Stack column-major matrices for the entry point (torch row-major view:
    element [j, c, r] = row r of column c)."""
    A = dev(np.stack([a.T for a in As]))
    Bm = dev(np.stack([b.T for b in Bs]))
    C, flags = h.block_pencils(A, Bm, q, has_p, tol)
    C = C.cpu().numpy()
    nS = (3 if has_p else 2) * q
    return [C[j].T[:nS] for j in range(len(As))], flags.cpu().numpy()


def theta_of(C, A):
    return np.real(np.einsum("it,ij,jt->t", C.conj(), A, C))


@pytest.mark.parametrize("q", [1, 2, 4, 8, 16, 20, 32])
@pytest.mark.parametrize("has_p", [True, False])
@pytest.mark.parametrize("cplx", [False, True])
def test_block_pencils_match_oracle(h64, q, has_p, cplx):
    rng = np.random.default_rng(100 * q + 10 * has_p + cplx)
    nS = (3 if has_p else 2) * q
    pens = [rand_pencil(nS, cplx, rng) for _ in range(3)]
    Cs, flags = gpu_pencils(h64, [a for a, _ in pens], [b for _, b in pens], q, has_p)
    for (A, Bm), C, f in zip(pens, Cs, flags):
        r = dense.block_pencil(A, Bm, q, has_p)
        th = theta_of(C, A)
        scale = np.abs(r.theta).max()
        err = np.abs(th - r.theta).max() / scale
        say("pencil q", q, "P", has_p, "cplx", cplx, "flags", hex(f), "theta err", err)
        assert err <= 1e-12
        assert bool(f & 1) == r.used_p and not (f & 2) and not (f & 4)
        assert (f >> 8) == r.dropped
        np.testing.assert_allclose(C.conj().T @ Bm @ C, np.eye(q), atol=1e-11)
        np.testing.assert_allclose(A @ C, Bm @ C * th[None, :], atol=1e-10 * np.abs(A).max())


@pytest.mark.parametrize("cplx", [False, True])
@pytest.mark.parametrize("p_low", [(-10.0, -9.0), (-10.0, 10.0)], ids=["CX-zero", "CX-rank1"])
def test_block_pencils_backtrack(h64, cplx, p_low):
    """C_X of the q lowest pairs is singular: the kernel re-solves without P
    (flag bit 1), like the oracle, and the P rows of C are zero."""
    rng = np.random.default_rng(7 + cplx)
    q = 2
    A, Bm = op_pencil(cplx, np.array(p_low), rng, q)
    r = dense.block_pencil(A, Bm, q, True)
    assert r.backtracked
    (C,), (f,) = gpu_pencils(h64, [A], [Bm], q, True)
    say("backtrack pencil", p_low, "flags", hex(f))
    assert f & 2 and not f & 1 and not f & 4
    assert np.all(C[2 * q:] == 0)
    th = theta_of(C, A)
    assert np.abs(th - r.theta).max() / np.abs(r.theta).max() <= 1e-12
    np.testing.assert_allclose(C.conj().T @ Bm @ C, np.eye(q), atol=1e-11)
    # the 2q x 2q solution the re-solve must equal
    (C2,), _ = gpu_pencils(h64, [A[:2 * q, :2 * q]], [Bm[:2 * q, :2 * q]], q, False)
    np.testing.assert_allclose(C[:2 * q], C2, atol=1e-12 * np.abs(C2).max())


@pytest.mark.parametrize("cplx", [False, True])
def test_block_pencils_singular_tol(cplx):
    """A weak X-P coupling: C_X small but nonsingular.  Kept with P at the
    default floor; solved without P when options.singular_tol exceeds every
    Cholesky pivot of C_X^H C_X -- as the oracle at the same floors."""
    rng = np.random.default_rng(41 + cplx)
    q = 2
    A, Bm = op_pencil(cplx, np.array([-10.0, -9.0]), rng, q, eps=1e-2)
    r = dense.block_pencil(A, Bm, q, True)
    Cx = r.C[:q]
    ev = np.linalg.eigvalsh(dense.sym(Cx.conj().T @ Cx))
    assert r.used_p and 1e-12 < ev.min() and ev.max() < 1e-2
    for stol, back in ((0.0, False), (2 * ev.max(), True), (ev.min() / 2, False)):
        h = B.Handle("fp64", singular_tol=stol)
        (C,), (f,) = gpu_pencils(h, [A], [Bm], q, True)
        ro = dense.block_pencil(A, Bm, q, True, singular_tol=stol if stol > 0 else dense.PIVOT_TOL)
        say("singular_tol", stol, "flags", hex(f), "oracle backtracked", ro.backtracked)
        assert bool(f & 2) == back == ro.backtracked
        th = theta_of(C, A)
        assert np.abs(th - ro.theta).max() / np.abs(ro.theta).max() <= 1e-12
        h.close()


def gpu_solve(h, p, tol=None, X0="default"):
    g = p.grid
    x0 = p.start() if isinstance(X0, str) else X0
    lam, X, info = h.solve(dev(p.V), g.N, p.k, p.q, tol or p.tol, p.rr_period,
                           None if x0 is None else dev(x0), h=g.h, order=g.order, kpt=g.kpt)
    return lam.cpu().numpy(), X.cpu().numpy(), info


def oracle_solve(p, tol=None, X0=None, **kw):
    g = p.grid
    A = lambda X: stencil.apply_h(X, p.V, g.N, g.h, g.order, g.kpt)
    T = 1.0 / stencil.diag_h(p.V, g.h, g.order)
    return ppcg_ref.ppcg(A, T, p.start() if X0 is None else X0, p.k, p.q, tol or p.tol, p.rr_period, **kw)


def laplacian_spectrum(N, h, order):
    th = 2 * np.pi * np.arange(N) / N
    s = 2.0 * np.sin(th / 2) ** 2 / h ** 2 if order == 2 else 0.5 * (30 - 32 * np.cos(th) + 2 * np.cos(2 * th)) / (
        12 * h ** 2)
    return np.sort((s[:, None, None] + s[None, :, None] + s[None, None, :]).ravel())


def test_solve_with_backtracks_matches_oracle():
    """singular_tol 0.9: the large early steps re-solve their blocks without
    P; GPU and oracle both backtrack and reach the dense eigenvalues."""
    p = I.small_problem(N=8, k=12, q=4, order=2, tol=1e-9)
    h = B.Handle("fp64", max_iter=MAX_IT, singular_tol=0.9)
    lam, X, info = gpu_solve(h, p)
    lo, Xo, io = oracle_solve(p, singular_tol=0.9)
    lb = brute.lowest_values(p.V, 8, 0.5, 2, p.k)
    scale = np.abs(lb).max()
    say("backtracks gpu/oracle", info["n_backtrack"], io.n_backtrack, "iters", info["iters"], io.iters)
    assert info["n_backtrack"] > 0 and io.n_backtrack > 0
    assert np.abs(lam - lo).max() / scale <= 1e-9
    assert np.abs(lam - lb).max() / scale <= 1e-9
    np.testing.assert_allclose(X.T @ X, np.eye(p.k), atol=1e-12)
    h.close()


UNLOCK_CASES = [dict(N=8, k=16, q=4, seed=1, rr_period=5), dict(N=6, k=12, q=4, seed=1, rr_period=2),
                dict(N=6, k=8, q=2, seed=3, rr_period=5), dict(N=6, k=12, q=2, seed=3, rr_period=1),
                dict(N=6, k=16, q=1, seed=2, rr_period=1)]


def test_solve_locked_set_shrinks(h64):
    """V = 0 with k inside a degenerate shell: soft locking re-decides the
    locked prefix at every Rayleigh-Ritz and it can shrink (P reset).  Every
    case gives the closed-form spectrum; the shrink happens on the GPU in at
    least one of them (in the oracle it happens in each)."""
    shrinks = 0
    for c in UNLOCK_CASES:
        p = I.small_problem(nwells=0, tol=1e-8, **c)
        lam, X, info = gpu_solve(h64, p)
        ex = laplacian_spectrum(p.grid.N, 0.5, 2)[:p.k]
        say("unlock case", c, "gpu n_unlock", info["n_unlock"], "iters", info["iters"])
        assert np.abs(lam - ex).max() <= 1e-9 * np.abs(ex).max()
        shrinks += info["n_unlock"]
    assert shrinks >= 1


def test_solve_exact_eigenvector_start(h64):
    p = I.small_problem(N=8, k=7, q=2, nwells=0, tol=1e-9)
    X0 = p.start()
    X0[:, 0] = 1.0
    lam, X, info = gpu_solve(h64, p, X0=X0)
    ex = laplacian_spectrum(8, 0.5, 2)[:7]
    say("exact eigenvector start: dropped", info["n_dropped"], "iters", info["iters"])
    assert info["n_dropped"] > 0
    assert np.abs(lam - ex).max() <= 1e-10


@pytest.mark.parametrize("kpt", [(0.0, 0.0, 0.0), (0.7, 0.0, 0.0)], ids=["real", "bloch"])
def test_start_block_drawn_on_device(kpt):
    """X0 = NULL: a seeded N(0,1) block from the device generator; the same
    seed repeats bit for bit, another seed reaches the same eigenvalues."""
    p = I.small_problem(N=8, k=12, q=4, order=2, tol=1e-9, kpt=kpt)
    lb = brute.lowest_values(p.V, 8, 0.5, 2, p.k, kpt)
    res = []
    for seed in (5, 5, 6):
        h = B.Handle("fp64", max_iter=MAX_IT, seed=seed)
        res.append(gpu_solve(h, p, X0=None))
        h.close()
    assert np.array_equal(res[0][0], res[1][0]) and np.array_equal(res[0][1], res[1][1])
    for lam, X, info in res:
        assert np.abs(lam - lb).max() / np.abs(lb).max() <= 1e-9
        assert info["resid_final"] <= 1e-9
    assert not np.array_equal(res[0][1], res[2][1])


@pytest.mark.parametrize("cplx", [False, True], ids=["real", "complex"])
def test_device_start_block_matches_oracle_generator(cplx):
    """ppcg_start_block against the oracle's Philox-4x32-10 + Box-Muller
    block, entry by entry: ragged row counts, a seed with a nonzero high
    word, empty blocks.  The uniforms are exact integer maps on both sides;
    log, sqrt and cos/sincospi differ by a few ulps, so |d - o| <= 3e-14 +
    1e-14 |o| (entries are below 8.7 in magnitude).  Then a solve with
    X0 = NULL equals, bit for bit, the solve given that block."""
    h = B.Handle("fp64", max_iter=MAX_IT, seed=11)
    for n, ncols, seed in ((1000, 7, 203), (777, 3, (1 << 40) + 5), (0, 3, 1), (5, 0, 1)):
        Xd = h.start_block(n, ncols, seed, cplx).cpu().numpy().T
        Xo = rng.start_block(n, ncols, seed, cplx)
        assert Xd.shape == Xo.shape == (n, ncols)
        err = np.abs(Xd - Xo)
        say("start block", n, ncols, seed, "max |d - o|", err.max() if err.size else 0.0)
        assert np.all(err <= 3e-14 + 1e-14 * np.abs(Xo))
    kpt = (0.7, 0.0, 0.0) if cplx else (0.0, 0.0, 0.0)
    p = I.small_problem(N=8, k=12, q=4, order=2, tol=1e-9, kpt=kpt)
    K = h.columns(p.k, p.q)
    X0 = h.start_block(p.grid.n, K, 11, cplx).cpu().numpy().T
    a = gpu_solve(h, p, X0=None)
    b = gpu_solve(h, p, X0=X0)
    h.close()
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_unpreconditioned_solve_matches_oracle(prec):
    """precond = PPCG_PRECOND_NONE (T = I in step 8 of Algorithm 3): the GPU
    against the oracle run with T = 1 and against the dense eigenvalues.
    With T = I a potential that makes diag(H) negative everywhere is solved
    (the spectrum shifts with it), where the Jacobi preconditioner reports
    PPCG_ENOTHPD; an unknown preconditioner value is PPCG_EINVAL."""
    p = I.small_problem(N=8, k=12, q=4, order=2, tol=1e-9)
    g = p.grid
    tol_l = 1e-9 if prec == "fp64" else 1e-7
    h = B.Handle(prec, max_iter=MAX_IT)

    def solve(V, **kw):
        lam, X, info = h.solve(dev(V), g.N, p.k, p.q, p.tol, p.rr_period, dev(p.start()), h=g.h, order=g.order, **kw)
        return lam.cpu().numpy(), X.cpu().numpy(), info

    lam, X, info = solve(p.V, precond="none")
    A = lambda Y: stencil.apply_h(Y, p.V, g.N, g.h, g.order, g.kpt)
    lo, Xo, io = ppcg_ref.ppcg(A, np.ones(g.n), p.start(), p.k, p.q, p.tol, p.rr_period)
    lj, _, ij = solve(p.V)
    lb = brute.lowest_values(p.V, 8, 0.5, 2, p.k)
    scale = np.abs(lb).max()
    say(prec, "T = I iters gpu", info["iters"], "oracle", io.iters, "| Jacobi iters gpu", ij["iters"])
    assert np.abs(lo - lb).max() / scale <= 1e-9
    assert np.abs(lam - lb).max() / scale <= tol_l
    assert np.abs(lam - lo).max() / scale <= tol_l
    assert info["resid_final"] <= p.tol
    np.testing.assert_allclose(X.T @ X, np.eye(p.k), atol=1e-12)
    Vneg = p.V - 14.0   # diag(H) = 12 + V < 0 at every point
    ln, _, infon = solve(Vneg, precond="none")
    assert np.abs(ln - (lb - 14.0)).max() / np.abs(lb - 14.0).max() <= tol_l
    with pytest.raises(B.PPCGError) as e:
        solve(Vneg, precond="jacobi")
    assert e.value.status == "PPCG_ENOTHPD"
    with pytest.raises(B.PPCGError) as e:
        solve(p.V, precond=7)
    assert e.value.status == "PPCG_EINVAL"
    h.close()


def test_tune_table_persists(tmp_path):
    """options.tune_table: the first tuned solve writes its decisions; a new
    handle reads them (no re-timing, same plans: the same bits)."""
    path = str(tmp_path / "tune.txt")
    p = I.small_problem(N=16, k=120, q=8, order=4, tol=1e-9)
    h1 = B.Handle("fp64", max_iter=MAX_IT, autotune=True, tune_table=path)
    a = gpu_solve(h1, p)
    b = gpu_solve(h1, p)
    lines = [ln for ln in open(path) if not ln.startswith("#")]
    say("tune table lines", len(lines))
    assert len(lines) >= 3
    mtime = os.path.getmtime(path)
    h2 = B.Handle("fp64", max_iter=MAX_IT, autotune=True, tune_table=path)
    c = gpu_solve(h2, p)
    assert "(from table)" in h2.tune_report()
    assert np.array_equal(b[0], c[0]) and np.array_equal(b[1], c[1])
    assert os.path.getmtime(path) == mtime
    h1.close()
    h2.close()
    bad = tmp_path / "bad.txt"
    bad.write_text("0 1 2 not a table\n")
    with pytest.raises(B.PPCGError) as e:
        B.Handle("fp64", autotune=True, tune_table=str(bad))
    assert e.value.status == "PPCG_EINVAL"


def test_iteration_log_and_stage_times():
    """The per-iteration log and the per-stage device times of a profiled
    solve; GPU and oracle residual histories are printed side by side (the
    iteration counts themselves have no pin)."""
    p = I.small_problem(N=10, k=20, q=4, order=4, tol=1e-9)
    log = []
    h = B.Handle("fp64", max_iter=MAX_IT, profile=True, log=log.append)
    lam, X, info = gpu_solve(h, p)
    io = oracle_solve(p, record=True)[2]
    say("iters gpu/oracle", info["iters"], io.iters)
    for i in range(0, max(len(log), len(io.history)), 10):
        g = log[i]["rho"] if i < len(log) else float("nan")
        o = io.history[i] if i < len(io.history) else float("nan")
        say(f"  iter {i:4d}  rho gpu {g:.6e}  oracle {o:.6e}")
    assert log[0]["iter"] == 0 and log[0]["kind"] == "start"
    assert [r["iter"] for r in log[:5]] == [0, 1, 2, 3, 4]
    assert log[-1]["rho"] <= p.tol
    # every Rayleigh-Ritz but the last (the final one that passed) ends an iteration in the log
    assert sum(r["kind"] in ("rr", "final_rr_failed") for r in log) + 1 == info["n_rr"]
    st = info["stage_ms"]
    kt = h.kernel_times()
    total = sum(v[0] for v in kt.values())
    say("stage ms", [round(x, 3) for x in st], "kernel total", round(total, 3), "roofline ms",
        info["roofline_ms"], "solve s", info["time_s"])
    assert st[1] > 0 and st[2] > 0 and st[3] > 0 and st[4] > 0
    assert abs(sum(st) - total) <= 1e-6 * total + 1e-9
    assert 0 < info["roofline_ms"] < 1e3 * info["time_s"]
    h.close()


def test_grad_reports_noconvergence():
    """ppcg_grad returns PPCG_ENOCONV with the residual when block CG stops
    at max_iter above tol, and PPCG_OK with a residual below tol otherwise."""
    p = I.small_problem(N=10, k=12, q=4, order=2, tol=1e-10)
    h = B.Handle("fp64", max_iter=MAX_IT)
    gpu_solve(h, p)
    g = dev(np.ones(p.k))
    w = dev(np.random.default_rng(3).standard_normal(p.grid.n))
    with pytest.raises(B.PPCGError) as e:
        h.grad(g, w, tol=1e-12, max_iter=2)
    assert e.value.status == "PPCG_ENOCONV" and e.value.info["resid"] > 1e-12
    dV, its = h.grad(g, w, tol=1e-10)
    say("grad iters", its, "resid", h.grad_resid)
    assert h.grad_resid <= 1e-10 and its > 2
    h.close()


def test_apply_h_rejects_bad_grid(h64):
    V = dev(np.zeros(27))
    X = dev(np.zeros((2, 27)))
    with pytest.raises(B.PPCGError) as e:
        h64.apply_h(V, 3, X)
    assert e.value.status == "PPCG_EINVAL"
    V4 = dev(np.zeros(64))
    with pytest.raises(B.PPCGError) as e:
        h64.apply_h(V4, 4, dev(np.zeros((1, 64))), h=0.0)
    assert e.value.status == "PPCG_EINVAL"
