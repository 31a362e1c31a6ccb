"""Batched solve (ppcg_solve_batched): many uneven problems in lockstep
through grouped launches, against separate single solves and dense brute
force.  Batched and single solves run the same arithmetic per problem; they
may differ in the number of row splits of a Gram (the single-solve handle
reuses one partial buffer across problem sizes), i.e. in rounding order."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from oracle import brute  # noqa: E402
from paper_1407_7506_amd import binding as B  # noqa: E402
from paper_1407_7506_amd import inputs as I  # noqa: E402

# iteration cap of every handle here: a solve that stops converging ends
# with PPCG_ENOCONV in seconds instead of running 20000 iterations
MAX_IT = 4000


def say(*a):
    print(*a, flush=True)


def dev(a):
    return torch.tensor(np.ascontiguousarray(a), device="cuda")


def small_batch():
    specs = [(8, 12, 2), (10, 20, 4), (9, 14, 4), (12, 30, 2), (8, 6, 2), (11, 24, 4)]
    out = []
    for i, (N, k, order) in enumerate(specs):
        p = I.small_problem(N=N, k=k, q=2, order=order, nwells=1 + i % 3, seed=50 + i, tol=1e-9)
        out.append(p)
    return out


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_batched_equals_single_solves(precision):
    ps = small_batch()
    h = B.Handle(precision, max_iter=MAX_IT)
    probs = [dict(V=dev(p.V), N=p.grid.N, k=p.k, X0=dev(p.start()), order=p.grid.order) for p in ps]
    res = h.solve_batched(probs, 2, 1e-9, 5)
    hs = B.Handle(precision, max_iter=MAX_IT)
    for p, pr, (lam, X, info, status) in zip(ps, probs, res):
        assert status == "PPCG_OK"
        l1, X1, i1 = hs.solve(pr["V"], pr["N"], p.k, 2, 1e-9, 5, pr["X0"], order=pr["order"])
        d = ((lam - l1).abs().max() / l1.abs().max()).item()
        say(p.name, "iters batched/single", info["iters"], i1["iters"], "max rel diff", d)
        assert d <= 1e-12
        lb, _, _ = brute.lowest(p.V, p.grid.N, 0.5, p.grid.order, p.k)
        assert np.abs(lam.cpu().numpy() - lb).max() / np.abs(lb).max() <= 1e-9


def test_batched_reports_per_problem_errors():
    ps = small_batch()[:3]
    h = B.Handle("fp64", max_iter=MAX_IT)
    probs = [dict(V=dev(p.V), N=p.grid.N, k=p.k, X0=dev(p.start()), order=p.grid.order) for p in ps]
    probs[1]["V"] = dev(np.full(ps[1].grid.n, -50.0))       # diag(H) < 0: not HPD
    res = h.solve_batched(probs, 2, 1e-8, 5, check=False)
    assert [r[3] for r in res] == ["PPCG_OK", "PPCG_ENOTHPD", "PPCG_OK"]


def test_batch64_workload_subset():
    """Eight problems of the 64-problem uneven workload (grids 24^3..40^3,
    k 32..256, sbsize 8) batched vs single solves."""
    ps = I.batch64()[:8]
    h = B.Handle("fp64", max_iter=MAX_IT)
    probs = [dict(V=dev(p.V), N=p.grid.N, k=p.k, X0=dev(p.start()), order=2) for p in ps]
    res = h.solve_batched(probs, 8, 1e-6, 5)
    hs = B.Handle("fp64", max_iter=MAX_IT)
    for p, pr, (lam, X, info, status) in zip(ps, probs, res):
        l1, X1, i1 = hs.solve(pr["V"], pr["N"], p.k, 8, 1e-6, 5, pr["X0"])
        d = ((lam - l1).abs().max() / l1.abs().max()).item()
        say(p.name, "iters", info["iters"], i1["iters"], "resid", info["resid_final"], "diff", d)
        assert status == "PPCG_OK" and info["resid_final"] <= 1e-6
        assert d <= 1e-9
