"""Warm-started PPCG over a sequence of slowly changing operators (the SCF
use of the method, section 6 of the paper): the first operator is solved to
tol from the given start block; every later one runs a fixed small number of
PPCG iterations (two in the paper's SCF runs) without Cholesky-QR, starting
from all K Ritz vectors (buffer vectors included) of the previous step.

Control flow and argument marshalling only: each step is one ppcg_solve
through the C ABI (options: PPCG_RETURN_BUFFERS, max_iter, orth)."""
from __future__ import annotations

from . import binding


def solve_sequence(Vs, N, k, sbsize, tol, rr_period, X0, *, precision="fp64", h=0.5, order=2, kpt=(0.0, 0.0, 0.0),
                   iters_per_step=2, first_max_iter=20000, orth="none", stream=None, log=None):
    """Vs: list of potentials (CUDA float64, N^3 each); X0: (n, K) start
    block of the first solve.  Returns ([(lam (k,), info dict) per step],
    X (n, K) Ritz vectors of the last step).  A later step's status is
    PPCG_OK when it met tol within iters_per_step iterations and
    PPCG_ENOCONV otherwise; both hold the final Rayleigh-Ritz pairs."""
    first = binding.Handle(precision, max_iter=first_max_iter, return_buffers=True, stream=stream)
    step = binding.Handle(precision, max_iter=iters_per_step, return_buffers=True, orth=orth, stream=stream,
                          log=log)
    try:
        lam, X, info = first.solve(Vs[0], N, k, sbsize, tol, rr_period, X0, h=h, order=order, kpt=kpt)
        out = [(lam[:k], info)]
        for V in Vs[1:]:
            lam, X, info = step.solve(V, N, k, sbsize, tol, rr_period, X, h=h, order=order, kpt=kpt, check=False)
            if info["status"] not in ("PPCG_OK", "PPCG_ENOCONV"):
                raise binding.PPCGError(binding.STATUS_CODE[info["status"]], step.error(), info)
            out.append((lam[:k], info))
        return out, X
    finally:
        first.close()
        step.close()
