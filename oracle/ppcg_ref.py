"""The PPCG iteration, step by step (oracle; test infrastructure).

Follows the paper's detailed algorithm (Algorithm 3, appendix) with the
practical aspects of section 5: block updates (5.1), the relative subspace
residual (5.2), buffer vectors (5.3), projections of W and P (5.4),
Cholesky-QR (5.5), periodic Rayleigh-Ritz (5.6) and soft locking (5.7).

Readings of places where the paper is silent or ambiguous:
  * the start block is orthonormalised by Cholesky-QR (the paper assumes an
    orthonormal X0);
  * in the per-block problem the q_j smallest pairs are kept (the algorithm
    box says k, the block-formulation text says k_j);
  * the Rayleigh-Ritz branch replaces Cholesky-QR in that iteration; the
    first Rayleigh-Ritz happens at iter = rr_period (iter starts at 1);
  * convergence: rho^2 = (sum over locked wanted columns of |w_i|^2 from the
    last Rayleigh-Ritz + |W_act(wanted)|_F^2) / (sum over locked wanted of
    lambda_i^2 + |G_act(wanted, wanted)|_F^2), wanted = the k leading columns;
    once rho <= tol, a final Rayleigh-Ritz is done and the residual of the k
    lowest Ritz pairs is recomputed from a fresh H X; iteration continues if
    that fails;
  * locking: the leading contiguous run of wanted Ritz vectors whose residual
    norm is at most tol * |Lambda_k|_F / (2 sqrt(k)), its length rounded down
    to a multiple of sbsize; re-decided at every Rayleigh-Ritz;
  * P is not rotated by the Rayleigh-Ritz; P(J_act) keeps the columns of the
    still-active absolute indices, and P is reset when the locked set shrinks;
  * H X, H W, H P are recomputed by the operator instead of being carried by
    recurrences (same quantities in exact arithmetic).
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

from . import dense
from .dense import RankError, block_pencil, cholqr, rayleigh_ritz, sym


class NoConvergence(RuntimeError):
    def __init__(self, msg, lam, X, info):
        super().__init__(msg)
        self.lam, self.X, self.info = lam, X, info


@dataclasses.dataclass
class Info:
    iters: int = 0
    n_rr: int = 0
    n_locked: int = 0
    rho: float = math.inf
    fresh_resid: float = math.inf
    history: list = dataclasses.field(default_factory=list)
    n_backtrack: int = 0      # sub-block solves redone without P (Theorem 1 test, Theorem 2)
    n_p_dropped: int = 0      # sub-blocks whose P columns were all dropped as dependent
    n_dropped: int = 0        # W/P columns left out of sub-block pencils (zero or dependent)
    n_unlock: int = 0         # Rayleigh-Ritz steps at which the locked set shrank (P reset)
    n_cholqr: int = 0         # non-RR iterations orthonormalised by Cholesky-QR
    n_taylor: int = 0         # ... by the Taylor polar step
    n_orth_skip: int = 0      # ... left as they were (steps 18-19 omitted)
    rr_iters: list = dataclasses.field(default_factory=list)   # iterations that ended with a Rayleigh-Ritz
    trace: float = math.nan   # trace of X^H A X over all K columns at the last loop head


def _fro2(M):
    return float(np.vdot(M, M).real) if M.size else 0.0


ORTH = ("cholqr", "skip", "taylor", "none")


def rr_schedule(rr_period, rr_max):
    """Iterations that end with a Rayleigh-Ritz step.  Fixed (rr_max <= rr_period):
    every rr_period-th iteration.  Dynamic (section 5.6: few Rayleigh-Ritz
    steps early, more once pairs converge and can be locked): the first after
    rr_max iterations, each following interval one shorter, down to rr_period."""
    it, gap = 0, max(rr_max, rr_period)
    while True:
        it += gap
        yield it
        gap = max(rr_period, gap - 1)


def ppcg(apply_a, tdiag, X0, k, sbsize, tol, rr_period, max_iter=20000, record=False,
         singular_tol=dense.PIVOT_TOL, orth="cholqr", orth_skip=0.1, orth_taylor=0.3, rr_max=0,
         stop="residual", bdiag=None):
    """Lowest k eigenpairs of the Hermitian operator ``apply_a`` (n x m -> n x m).

    tdiag : (n,) diagonal of the preconditioner T (Jacobi: 1/diag(H)), must be > 0.
    X0    : (n, K) start block, K = k + nbuf columns (buffer vectors included).
    singular_tol : floor of the Theorem 1 test on C_X (a block whose
            C_X^H C_X has a smaller Cholesky pivot is solved again without P).
    orth  : orthonormalisation of the updated block in iterations without a
            Rayleigh-Ritz step (steps 17-19; section 5.5), decided from
            e = |Xbar^H Xbar - I|_F over the active columns:
            "cholqr" always Cholesky-QR; "skip" omit steps 18-19 while
            e <= orth_skip, else Cholesky-QR; "taylor" omit while e <= orth_skip,
            the four-term Taylor polar step while e <= orth_taylor, else
            Cholesky-QR; "none" always omit them (the SCF use of section 6).
    rr_max : dynamic Rayleigh-Ritz period (see rr_schedule); 0 = fixed.
    stop  : "residual" -- relative subspace residual <= tol and the fresh
            residual check after the final Rayleigh-Ritz (section 5.2);
            "trace" -- relative change of trace(X^H A X) (all K columns)
            between consecutive loop heads below tol, then the final
            Rayleigh-Ritz without the fresh check (section 5.2).
    bdiag : (n,) positive diagonal of B for the generalized problem
            A x = lambda B x (section 1: the method carries over without
            factoring B): every inner product of the method becomes a B inner
            product -- X^H B X = I, residual A X - B X (X^H A X), projector
            I - X (B X)^H, sub-block and Rayleigh-Ritz Grams S^H B S.
            None: B = I.
    Returns (lam[:k] ascending, X[:, :k], Info).  Raises RankError on a
    Cholesky breakdown and NoConvergence after max_iter iterations.
    """
    n, K = X0.shape
    q = int(sbsize)
    if not (0 < k < K <= n) or q < 1 or tol <= 0 or rr_period < 1:
        raise ValueError("invalid PPCG arguments")
    tdiag = np.asarray(tdiag, dtype=np.float64)
    if np.any(~(tdiag > 0)):
        raise ValueError("preconditioner is not positive definite")
    if orth not in ORTH or stop not in ("residual", "trace"):
        raise ValueError("invalid orth or stop")
    if bdiag is not None:
        bdiag = np.asarray(bdiag, dtype=np.float64)
        if np.any(~(bdiag > 0)):
            raise ValueError("B is not positive definite")
    Bm = (lambda Y: Y) if bdiag is None else (lambda Y: bdiag[:, None] * Y)
    sched = rr_schedule(rr_period, rr_max)
    next_rr = next(sched)
    trace_prev = None
    info = Info()

    # steps 1-4: orthonormal start, residual W = AX - X (X^H A X)
    X0 = np.array(X0, dtype=np.result_type(X0.dtype, np.float64))
    X, _ = cholqr(X0, Bm(X0))
    nl = 0
    AXa = apply_a(X)
    G = sym(X.conj().T @ AXa)
    W = AXa - Bm(X) @ G
    P = None
    lock_wn = np.zeros(0)
    lock_lam = np.zeros(0)
    it = 1

    def rr_and_lock(X, nl, P):
        """Rayleigh-Ritz over [X, X_lock] then locking (RR branch)."""
        AS = apply_a(X)
        Xn, lam, _ = rayleigh_ritz(X, AS, Bm(X))
        AXn = apply_a(Xn)
        Wall = AXn - Bm(Xn) * lam[None, :]
        wn = np.sqrt(np.real(np.sum(Wall[:, :k].conj() * Wall[:, :k], axis=0)))
        fresh = math.sqrt(_fro2(Wall[:, :k])) / max(np.linalg.norm(lam[:k]), np.finfo(float).tiny)
        thr = 0.5 * tol * np.linalg.norm(lam[:k]) / math.sqrt(k)
        nl_new = 0
        while nl_new < k and wn[nl_new] <= thr:
            nl_new += 1
        nl_new = (nl_new // q) * q
        if P is not None:
            if nl_new < nl:
                info.n_unlock += 1
            P = P[:, nl_new - nl:] if nl_new >= nl else None
        return Xn, lam, AXn, Wall, wn, fresh, nl_new, P

    while True:
        m = K - nl
        nwa = max(0, k - nl)
        num = float(np.sum(lock_wn ** 2)) + _fro2(W[:, :nwa])
        den = float(np.sum(lock_lam ** 2)) + _fro2(G[:nwa, :nwa])
        rho = math.sqrt(num / den) if den > 0 else math.inf
        info.rho = rho
        trace = float(np.sum(lock_lam)) + float(np.real(np.trace(G)))
        info.trace = trace
        if record:
            info.history.append(rho)
        if stop == "trace":
            done = trace_prev is not None and abs(trace - trace_prev) <= tol * abs(trace)
            trace_prev = trace
        else:
            done = rho <= tol
        if done:
            # final Rayleigh-Ritz (steps 22-24) and a fresh residual check
            X, lam, AXn, Wall, wn, fresh, nl, P = rr_and_lock(X, nl, P)
            info.n_rr += 1
            info.fresh_resid = fresh
            if fresh <= tol or stop == "trace":
                info.iters = it - 1
                info.n_locked = nl
                info.X_all, info.lam_all = X, lam
                return lam[:k].copy(), X[:, :k].copy(), info
            lock_wn, lock_lam = wn[:nl], lam[:nl]
            W, G = Wall[:, nl:], np.diag(lam[nl:]).astype(X.dtype)
            AXa = AXn[:, nl:]
            continue
        if it > max_iter:
            info.iters = it - 1
            info.n_locked = nl
            X2, lam, _ = rayleigh_ritz(X, apply_a(X), Bm(X))
            info.X_all, info.lam_all = X2, lam
            raise NoConvergence("max_iter reached", lam[:k], X2[:, :k], info)

        XL = X[:, :nl]
        Xa = X[:, nl:]
        # step 8: precondition
        W = tdiag[:, None] * W
        # step 9: W <- (I - X X^H) W, then (I - X_lock X_lock^H) W
        # (generalized problem: the B-orthogonal projector I - X (B X)^H)
        BXa, BXL = Bm(Xa), Bm(XL)
        W = W - Xa @ (BXa.conj().T @ W)
        if nl:
            W = W - XL @ (BXL.conj().T @ W)
        # step 10: same for P
        if P is not None:
            P = P - Xa @ (BXa.conj().T @ P)
            if nl:
                P = P - XL @ (BXL.conj().T @ P)
        AW = apply_a(W)
        AP = apply_a(P) if P is not None else None
        # steps 11-16: independent projected problems per sub-block
        s = -(-m // q)
        Xbar = np.empty_like(Xa)
        Pn = np.empty_like(W)
        for j in range(s):
            c0, c1 = j * q, min(m, (j + 1) * q)
            blocks = [Xa[:, c0:c1], W[:, c0:c1]]
            ablocks = [AXa[:, c0:c1], AW[:, c0:c1]]
            if P is not None:
                blocks.append(P[:, c0:c1])
                ablocks.append(AP[:, c0:c1])
            S = np.concatenate(blocks, axis=1)
            AS = np.concatenate(ablocks, axis=1)
            Aj = sym(S.conj().T @ AS)
            Bj = sym(S.conj().T @ Bm(S))
            nx = c1 - c0
            res = block_pencil(Aj, Bj, nx, P is not None, singular_tol=singular_tol)
            C = res.C
            info.n_dropped += res.dropped
            if res.backtracked:
                info.n_backtrack += 1
            elif P is not None and not res.used_p:
                info.n_p_dropped += 1
            Cx, Cw = C[:nx], C[nx:2 * nx]
            Pj = W[:, c0:c1] @ Cw
            if P is not None:
                Pj = Pj + P[:, c0:c1] @ C[2 * nx:3 * nx]
            Pn[:, c0:c1] = Pj
            Xbar[:, c0:c1] = Xa[:, c0:c1] @ Cx + Pj
        P = Pn
        if it != next_rr:
            # steps 17-20: orthonormalise (or not, section 5.5), new residual
            G1 = sym(Xbar.conj().T @ Bm(Xbar))
            e = float(np.linalg.norm(G1 - np.eye(G1.shape[0])))
            if orth == "none" or (orth in ("skip", "taylor") and e <= orth_skip):
                Xa = Xbar
                info.n_orth_skip += 1
            elif orth == "taylor" and e <= orth_taylor:
                Xa = dense.polar_taylor(Xbar, G1)
                info.n_taylor += 1
            else:
                Xa, _ = cholqr(Xbar, Bm(Xbar))
                info.n_cholqr += 1
            X = np.concatenate([XL, Xa], axis=1)
            AXa = apply_a(Xa)
            G = sym(Xa.conj().T @ AXa)
            W = AXa - Bm(Xa) @ G
        else:
            # steps 21-31: Rayleigh-Ritz over [X, X_lock], then locking
            X = np.concatenate([XL, Xbar], axis=1)
            X, lam, AXn, Wall, wn, fresh, nl, P = rr_and_lock(X, nl, P)
            info.n_rr += 1
            info.rr_iters.append(it)
            next_rr = next(sched)
            lock_wn, lock_lam = wn[:nl], lam[:nl]
            W, G = Wall[:, nl:], np.diag(lam[nl:]).astype(X.dtype)
            AXa = AXn[:, nl:]
        it += 1
